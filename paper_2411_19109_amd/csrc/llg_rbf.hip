// Level-set function from radial basis functions and the Adam update of their
// amplitudes.
//
// Eq. 2: RBF i is the multiquadric cone g_i(x, y) = s_i - sqrt((x - x_i)^2 +
// (y - y_i)^2 + c^2).  Eq. 3: the level set is the shifted p-norm of the cones,
// Phi = [sum_i (g_i + dphi)^p]^(1/p) - dphi, with dphi the absolute value of the
// smallest cone value on the design region; Phi is then renormalised to
// [-1, 1] by its largest magnitude on the design region (the paragraph after
// Eq. 3).  Coordinates are node indices.  Outside the design region Phi = 0.
//
// Forward, per node of the design region:
//   k_rbf_cones   pass 1 over the RBFs: the node's largest cone (kept for
//                 pass 2) and a block minimum of all cone values -> dphi;
//   k_rbf_pnorm   pass 2: S = gmax_b * (sum_i (b_i / gmax_b)^p)^(1/p) with
//                 b_i = g_i + dphi and gmax_b the largest base (scaling by the
//                 largest base keeps every power in [0, 1]: no overflow at
//                 p = 90 in either precision), Phi_raw = S - dphi, block max |Phi_raw|;
//   k_rbf_scale   Phi = Phi_raw / max |Phi_raw| on the design region, 0 elsewhere.
// The RBFs of a pass are staged in LDS in chunks and read by broadcast; a
// group of TPN adjacent lanes shares one node and splits its RBFs (butterfly
// combine), so that small grids still fill the chip.  TPN and every reduction
// order are fixed by the grid size alone: results are reproducible bit for bit.
//
// Backward (dphi and the scale held fixed): dJ/ds_i = scale * sum_x dJ/dPhi(x)
// ((g_i(x) + dphi) / S(x))^(p - 1).  Blocks tile (node chunk) x (group of RB
// RBFs held in registers); each writes per-chunk partial sums, which a second
// kernel adds in chunk order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "llg.h"
#include "llg_internal.hpp"

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 1024;  // RBFs staged in LDS per pass
constexpr int kRB = 4;        // RBFs per block of the backward kernel
constexpr int kMinBlocks = 1024;

template <typename T> struct RbfL { T x, y, s, pad; };

__device__ inline float vsqrt(float v) { return __builtin_sqrtf(v); }
__device__ inline double vsqrt(double v) { return __builtin_sqrt(v); }
__device__ inline float vlog2(float v) { return log2f(v); }
__device__ inline double vlog2(double v) { return log2(v); }
__device__ inline float vexp2(float v) { return exp2f(v); }
__device__ inline double vexp2(double v) { return exp2(v); }

// Eq. 2 at node (x, y).  One function for every pass, so that all passes see
// the same cone values.
template <typename T>
__device__ inline T cone(T x, T y, const RbfL<T>& r, T c2) {
    const T dx = x - r.x, dy = y - r.y;
    return r.s - vsqrt(dx * dx + dy * dy + c2);
}

struct OpMin { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpSum { __device__ double operator()(double a, double b) const { return a + b; } };

// Block-wide reduction in a fixed order (butterfly in each wave, then the
// waves in index order); every thread receives the result.
template <typename Op>
__device__ double block_reduce(double v, Op op, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int w = 1; w < kThreads / 64; ++w) r = op(r, sh[w]);
    return r;
}

template <typename T>
__device__ inline void stage_rbfs(RbfL<T>* R, const double* __restrict__ ctr, const double* __restrict__ s, int n,
                                  int b0, int m) {
    for (int i = threadIdx.x; i < m; i += kThreads)
        R[i] = RbfL<T>{(T)ctr[b0 + i], (T)ctr[n + b0 + i], (T)s[b0 + i], T(0)};
}

template <typename T, int TPN>
__global__ __launch_bounds__(kThreads) void k_rbf_cones(int nx, int nnode, int n, const double* __restrict__ ctr,
                                                        const double* __restrict__ s, T c2,
                                                        const uint8_t* __restrict__ design, T* __restrict__ gmax_out,
                                                        double* __restrict__ part_min) {
    __shared__ RbfL<T> R[kChunk];
    __shared__ double red[kThreads / 64];
    const int node = blockIdx.x * (kThreads / TPN) + threadIdx.x / TPN;
    const int sub = threadIdx.x % TPN;
    const bool act = node < nnode && design[node] != 0;
    const T x = (T)(node % nx), y = (T)(node / nx);
    T gmin = (T)INFINITY, gmax = -(T)INFINITY;
    for (int b0 = 0; b0 < n; b0 += kChunk) {
        const int m = min(kChunk, n - b0);
        __syncthreads();
        stage_rbfs(R, ctr, s, n, b0, m);
        __syncthreads();
        if (act) {
            for (int i = sub; i < m; i += TPN) {
                const T g = cone(x, y, R[i], c2);
                gmin = fmin(gmin, g);
                gmax = fmax(gmax, g);
            }
        }
    }
    for (int o = TPN / 2; o > 0; o >>= 1) {
        gmin = fmin(gmin, __shfl_xor(gmin, o));
        gmax = fmax(gmax, __shfl_xor(gmax, o));
    }
    if (act && sub == 0) gmax_out[node] = gmax;
    const double bm = block_reduce(act ? (double)gmin : (double)INFINITY, OpMin(), red);
    if (threadIdx.x == 0) part_min[blockIdx.x] = bm;
}

template <typename T, int TPN>
__global__ __launch_bounds__(kThreads) void k_rbf_pnorm(int nx, int nnode, int n, const double* __restrict__ ctr,
                                                        const double* __restrict__ s, T c2, T p,
                                                        const uint8_t* __restrict__ design,
                                                        const double* __restrict__ scal, T* __restrict__ phi,
                                                        T* __restrict__ S_out, double* __restrict__ part_max) {
    __shared__ RbfL<T> R[kChunk];
    __shared__ double red[kThreads / 64];
    const int node = blockIdx.x * (kThreads / TPN) + threadIdx.x / TPN;
    const int sub = threadIdx.x % TPN;
    const bool act = node < nnode && design[node] != 0;
    const T x = (T)(node % nx), y = (T)(node / nx);
    const T dphi = (T)scal[0];
    const T bmax = act ? phi[node] + dphi : T(0);  // largest base of this node (pass 1)
    const T inv = bmax > T(0) ? T(1) / bmax : T(0);
    T acc = T(0);
    for (int b0 = 0; b0 < n; b0 += kChunk) {
        const int m = min(kChunk, n - b0);
        __syncthreads();
        stage_rbfs(R, ctr, s, n, b0, m);
        __syncthreads();
        if (act) {
            for (int i = sub; i < m; i += TPN) {
                const T b = fmax(cone(x, y, R[i], c2) + dphi, T(0));
                acc += vexp2(p * vlog2(b * inv));
            }
        }
    }
    for (int o = TPN / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const T S = bmax > T(0) ? bmax * vexp2(vlog2(acc) / p) : T(0);
    const T raw = S - dphi;
    if (act && sub == 0) {
        phi[node] = raw;
        if (S_out) S_out[node] = S;
    }
    const double bm = block_reduce(act ? fabs((double)raw) : 0.0, OpMax(), red);
    if (threadIdx.x == 0) part_max[blockIdx.x] = bm;
}

// mode 0: scal[0] = dphi = |min of the partial minima| (0 for an empty design
// region); mode 1: scal[1] = 1 / max of the partial maxima (1 without
// renormalisation or when Phi vanishes on the design region).
__global__ __launch_bounds__(kThreads) void k_rbf_finish(const double* __restrict__ part, int nb, int mode,
                                                         int normalize, double* __restrict__ scal) {
    __shared__ double red[kThreads / 64];
    double v;
    if (mode == 0) {
        v = INFINITY;
        for (int i = threadIdx.x; i < nb; i += kThreads) v = fmin(v, part[i]);
        v = block_reduce(v, OpMin(), red);
        if (threadIdx.x == 0) scal[0] = isinf(v) ? 0.0 : fabs(v);
    } else {
        v = 0.0;
        for (int i = threadIdx.x; i < nb; i += kThreads) v = fmax(v, part[i]);
        v = block_reduce(v, OpMax(), red);
        if (threadIdx.x == 0) scal[1] = (normalize && v > 0.0) ? 1.0 / v : 1.0;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_rbf_scale(int nnode, const uint8_t* __restrict__ design,
                                                        const double* __restrict__ scal, T* __restrict__ phi) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= nnode) return;
    phi[i] = design[i] ? (T)((double)phi[i] * scal[1]) : T(0);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_rbf_vjp(int nx, int nnode, int n, const double* __restrict__ ctr,
                                                      const double* __restrict__ s, T c2, T pm1,
                                                      const uint8_t* __restrict__ design,
                                                      const double* __restrict__ dJdphi, const T* __restrict__ S,
                                                      const double* __restrict__ scal, int chunk,
                                                      double* __restrict__ part) {
    __shared__ double red[kThreads / 64];
    const int i0 = blockIdx.y * kRB;
    RbfL<T> r[kRB];
    for (int k = 0; k < kRB; ++k) {
        const int i = min(i0 + k, n - 1);
        r[k] = RbfL<T>{(T)ctr[i], (T)ctr[n + i], (T)s[i], T(0)};
    }
    const T dphi = (T)scal[0];
    double acc[kRB];
    for (int k = 0; k < kRB; ++k) acc[k] = 0.0;
    const int beg = blockIdx.x * chunk, end = min(beg + chunk, nnode);
    for (int node = beg + (int)threadIdx.x; node < end; node += kThreads) {
        const T Sx = S[node];
        if (!design[node] || !(Sx > T(0))) continue;
        const double w = dJdphi[node];
        const T inv = T(1) / Sx;
        const T x = (T)(node % nx), y = (T)(node / nx);
        for (int k = 0; k < kRB; ++k) {
            const T b = fmax(cone(x, y, r[k], c2) + dphi, T(0)) * inv;
            const T t = b > T(0) ? vexp2(pm1 * vlog2(b)) : (pm1 == T(0) ? T(1) : T(0));
            acc[k] += w * (double)t;
        }
    }
    for (int k = 0; k < kRB; ++k) {
        const double v = block_reduce(acc[k], OpSum(), red);
        if (threadIdx.x == 0 && i0 + k < n) part[(size_t)blockIdx.x * n + i0 + k] = v;
    }
}

__global__ __launch_bounds__(kThreads) void k_rbf_vjp_finish(int n, int nchunk, const double* __restrict__ part,
                                                             const double* __restrict__ scal,
                                                             double* __restrict__ dJds) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    double a = 0.0;
    for (int c = 0; c < nchunk; ++c) a += part[(size_t)c * n + i];
    dJds[i] = scal[1] * a;
}

// Adam (Kingma & Ba, Algorithm 1) with the bias corrections c1 = 1 - beta1^t,
// c2 = 1 - beta2^t computed on the host.
__global__ __launch_bounds__(kThreads) void k_adam(int n, double* __restrict__ s, const double* __restrict__ g,
                                                   double* __restrict__ m, double* __restrict__ v, double lr,
                                                   double b1, double b2, double eps, double c1, double c2) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    s[i] = s[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps);
}

// Launch shape, fixed by the sizes alone.
struct Plan {
    int tpn;     // lanes per node in the forward passes
    int nb;      // forward blocks
    int chunk;   // nodes per backward block
    int nchunk;  // backward node chunks
    int ngrp;    // backward RBF groups
};

Plan plan_of(long long nnode, int n) {
    Plan P;
    P.tpn = 1;
    while (P.tpn < 16 && (nnode * P.tpn + kThreads - 1) / kThreads < kMinBlocks) P.tpn *= 2;
    P.nb = (int)((nnode * P.tpn + kThreads - 1) / kThreads);
    P.ngrp = (n + kRB - 1) / kRB;
    long long want = std::max(1, (kMinBlocks + P.ngrp - 1) / P.ngrp);
    long long chunk = (nnode + want - 1) / want;
    chunk = (chunk + kThreads - 1) / kThreads * kThreads;
    P.chunk = (int)chunk;
    P.nchunk = (int)((nnode + chunk - 1) / chunk);
    return P;
}

long long work_len_of(const Plan& P, int n) { return 2 + 2LL * P.nb + (long long)P.nchunk * n; }

int check_common(int32_t dtype, int32_t nx, int32_t ny, int32_t n, double c, double p) {
    if (dtype != LLG_F32 && dtype != LLG_F64) return llg::set_error(LLG_EINVAL, "rbf: dtype must be LLG_F32 or LLG_F64");
    if (nx < 1 || ny < 1 || (long long)nx * ny > (1LL << 30))
        return llg::set_error(LLG_ESHAPE, "rbf: grid must have 1 <= nx*ny <= 2^30 nodes");
    if (n < 1 || n > (1 << 17)) return llg::set_error(LLG_EINVAL, "rbf: need 1 <= n_rbf <= 131072");
    if (!std::isfinite(c)) return llg::set_error(LLG_EINVAL, "rbf: c must be finite");
    if (!std::isfinite(p) || p < 1.0) return llg::set_error(LLG_EINVAL, "rbf: p must be finite and >= 1");
    return LLG_OK;
}

int hip_status(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        static thread_local char buf[256];
        snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
        return llg::set_error(LLG_EHIP, buf);
    }
    return LLG_OK;
}

template <typename T, int TPN>
void launch_fwd_passes(const Plan& P, int nx, int nnode, int n, const double* ctr, const double* s, T c2, T p,
                       const uint8_t* design, T* phi, T* S_out, double* work, hipStream_t st) {
    double* part_min = work + 2;
    double* part_max = work + 2 + P.nb;
    k_rbf_cones<T, TPN><<<P.nb, kThreads, 0, st>>>(nx, nnode, n, ctr, s, c2, design, phi, part_min);
    k_rbf_finish<<<1, kThreads, 0, st>>>(part_min, P.nb, 0, 0, work);
    k_rbf_pnorm<T, TPN><<<P.nb, kThreads, 0, st>>>(nx, nnode, n, ctr, s, c2, p, design, work, phi, S_out, part_max);
}

template <typename T>
int rbf_forward(const Plan& P, int nx, int nnode, int n, const double* ctr, const double* s, double c, double p,
                const uint8_t* design, int normalize, T* phi, T* S_out, double* work, hipStream_t st) {
    const T c2 = (T)(c * c), pp = (T)p;
    switch (P.tpn) {
        case 1: launch_fwd_passes<T, 1>(P, nx, nnode, n, ctr, s, c2, pp, design, phi, S_out, work, st); break;
        case 2: launch_fwd_passes<T, 2>(P, nx, nnode, n, ctr, s, c2, pp, design, phi, S_out, work, st); break;
        case 4: launch_fwd_passes<T, 4>(P, nx, nnode, n, ctr, s, c2, pp, design, phi, S_out, work, st); break;
        case 8: launch_fwd_passes<T, 8>(P, nx, nnode, n, ctr, s, c2, pp, design, phi, S_out, work, st); break;
        default: launch_fwd_passes<T, 16>(P, nx, nnode, n, ctr, s, c2, pp, design, phi, S_out, work, st); break;
    }
    k_rbf_finish<<<1, kThreads, 0, st>>>(work + 2 + P.nb, P.nb, 1, normalize, work);
    k_rbf_scale<T><<<(nnode + kThreads - 1) / kThreads, kThreads, 0, st>>>(nnode, design, work, phi);
    return hip_status("rbf level set launch");
}

template <typename T>
int rbf_backward(const Plan& P, int nx, int nnode, int n, const double* ctr, const double* s, double c, double p,
                 const uint8_t* design, const double* dJdphi, const T* S, const double* work, double* part,
                 double* dJds, hipStream_t st) {
    k_rbf_vjp<T><<<dim3(P.nchunk, P.ngrp), kThreads, 0, st>>>(nx, nnode, n, ctr, s, (T)(c * c), (T)(p - 1.0), design,
                                                              dJdphi, S, work, P.chunk, part);
    k_rbf_vjp_finish<<<(n + kThreads - 1) / kThreads, kThreads, 0, st>>>(n, P.nchunk, part, work, dJds);
    return hip_status("rbf level set VJP launch");
}

}  // namespace

extern "C" {

int llg_rbf_work_len(int32_t nx, int32_t ny, int32_t n_rbf, int64_t* len) {
    if (!len) return llg::set_error(LLG_EINVAL, "rbf: NULL argument");
    const int rc = check_common(LLG_F64, nx, ny, n_rbf, 0.0, 1.0);
    if (rc) return rc;
    *len = work_len_of(plan_of((long long)nx * ny, n_rbf), n_rbf);
    return LLG_OK;
}

int llg_rbf_levelset(int32_t dtype, int32_t nx, int32_t ny, int32_t n_rbf, const double* centers, const double* s,
                     double c, double p, const uint8_t* design, int normalize, void* phi_out, void* pnorm_out,
                     double* work, hipStream_t stream) {
    int rc = check_common(dtype, nx, ny, n_rbf, c, p);
    if (rc) return rc;
    if (!centers || !s || !design || !phi_out || !work) return llg::set_error(LLG_EINVAL, "rbf: NULL argument");
    const int nnode = nx * ny;
    const Plan P = plan_of(nnode, n_rbf);
    if (dtype == LLG_F32)
        return rbf_forward<float>(P, nx, nnode, n_rbf, centers, s, c, p, design, normalize, (float*)phi_out,
                                  (float*)pnorm_out, work, stream);
    return rbf_forward<double>(P, nx, nnode, n_rbf, centers, s, c, p, design, normalize, (double*)phi_out,
                               (double*)pnorm_out, work, stream);
}

int llg_rbf_levelset_vjp(int32_t dtype, int32_t nx, int32_t ny, int32_t n_rbf, const double* centers,
                         const double* s, double c, double p, const uint8_t* design, const double* dJdphi,
                         const void* pnorm, double* work, double* dJds_out, hipStream_t stream) {
    int rc = check_common(dtype, nx, ny, n_rbf, c, p);
    if (rc) return rc;
    if (!centers || !s || !design || !dJdphi || !pnorm || !work || !dJds_out)
        return llg::set_error(LLG_EINVAL, "rbf: NULL argument");
    const int nnode = nx * ny;
    const Plan P = plan_of(nnode, n_rbf);
    double* part = work + 2 + 2 * P.nb;
    if (dtype == LLG_F32)
        return rbf_backward<float>(P, nx, nnode, n_rbf, centers, s, c, p, design, dJdphi, (const float*)pnorm, work,
                                   part, dJds_out, stream);
    return rbf_backward<double>(P, nx, nnode, n_rbf, centers, s, c, p, design, dJdphi, (const double*)pnorm, work,
                                part, dJds_out, stream);
}

int llg_adam_step(int32_t n, double* s, const double* grad, double* m, double* v, int64_t t, double lr, double beta1,
                  double beta2, double eps, hipStream_t stream) {
    if (!s || !grad || !m || !v) return llg::set_error(LLG_EINVAL, "adam: NULL argument");
    if (n < 1 || t < 1) return llg::set_error(LLG_EINVAL, "adam: need n >= 1 and t >= 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.0) || !std::isfinite(lr))
        return llg::set_error(LLG_EINVAL, "adam: need 0 <= beta1, beta2 < 1, eps >= 0 and a finite lr");
    const double c1 = 1.0 - std::pow(beta1, (double)t), c2 = 1.0 - std::pow(beta2, (double)t);
    k_adam<<<(n + kThreads - 1) / kThreads, kThreads, 0, stream>>>(n, s, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    return hip_status("adam launch");
}

}  // extern "C"
