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
// RBFs held in registers); each thread sums its nodes in the map's precision,
// blocks reduce in float64 and write per-chunk partial sums, which a second
// kernel adds in chunk order.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <vector>

#include "llg.h"
#include "llg_internal.hpp"

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 1024;  // RBFs staged in LDS per pass
constexpr int kRB = 8;        // RBFs per block of the backward kernel
constexpr int kMinBlocks = 1024;

template <typename T> struct RbfL { T x, y, s, pad; };

// FP32: the hardware square root, base-2 logarithm and exponential (about 1
// ulp each).  Their arguments here are normal (sqrt sees d^2 + c^2 >= c^2 > 0)
// or harmlessly flushed: a ratio below 2^-126 enters as 0, whose power is 0
// (its true value, raised to p, is far below a sum that is at least 1).  FP64:
// the correctly rounded library functions.
__device__ inline float vsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ inline double vsqrt(double v) { return __builtin_sqrt(v); }
__device__ inline float vlog2(float v) { return __builtin_amdgcn_logf(v); }
__device__ inline double vlog2(double v) { return log2(v); }
__device__ inline float vexp2(float v) { return __builtin_amdgcn_exp2f(v); }
__device__ inline double vexp2(double v) { return exp2(v); }
__device__ inline float vrcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ inline double vrcp(double v) { return 1.0 / v; }

// Eq. 2 at node (x, y): r.s - sqrt(dx^2 + dy^2 + c^2).  The p-norm passes
// stage r.s = s_i + dphi, so that the same call gives the base g_i + dphi.
template <typename T>
__device__ inline T cone(T x, T y, const RbfL<T>& r, T c2) {
    const T dx = x - r.x, dy = y - r.y;
    return r.s - vsqrt(fma(dx, dx, fma(dy, dy, c2)));
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
                                  int b0, int m, T shift) {
    for (int i = threadIdx.x; i < m; i += kThreads)
        R[i] = RbfL<T>{(T)ctr[b0 + i], (T)ctr[n + b0 + i], (T)s[b0 + i] + shift, T(0)};
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
        stage_rbfs(R, ctr, s, n, b0, m, T(0));
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
        stage_rbfs(R, ctr, s, n, b0, m, dphi);
        __syncthreads();
        if (act) {
            for (int i = sub; i < m; i += TPN) {
                const T b = fmax(cone(x, y, R[i], c2), T(0));
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

// UNIT: p = 1, where every power (b/S)^(p-1) is 1 (also for b = 0).
template <typename T, bool UNIT>
__global__ __launch_bounds__(kThreads) void k_rbf_vjp(int nx, int nnode, int n, const double* __restrict__ ctr,
                                                      const double* __restrict__ s, T c2, T pm1,
                                                      const uint8_t* __restrict__ design,
                                                      const double* __restrict__ dJdphi, const T* __restrict__ S,
                                                      const double* __restrict__ scal, int chunk,
                                                      double* __restrict__ part) {
    __shared__ double red[kThreads / 64];
    const int i0 = blockIdx.y * kRB;
    const T dphi = (T)scal[0];
    RbfL<T> r[kRB];
    for (int k = 0; k < kRB; ++k) {
        const int i = min(i0 + k, n - 1);
        r[k] = RbfL<T>{(T)ctr[i], (T)ctr[n + i], (T)s[i] + dphi, T(0)};
    }
    T acc[kRB];
    for (int k = 0; k < kRB; ++k) acc[k] = T(0);
    const int beg = blockIdx.x * chunk, end = min(beg + chunk, nnode);  // beg < nnode: chunks cover the grid
    // node coordinates advance by kThreads nodes per iteration: qy rows and qx columns
    const int qy = kThreads / nx, qx = kThreads - qy * nx;
    int node = beg + (int)threadIdx.x;
    int iy = node / nx, ix = node - iy * nx;
    // A node's inputs are loaded one node ahead, unconditionally (the index is
    // clamped into the chunk), into two alternating register sets (the loop is
    // unrolled by two), so that no copy waits on a load in flight and the load
    // latency overlaps the previous node's arithmetic.
    const int last = max(end - 1, beg);
    auto visit = [&](T Sv, double wv, uint8_t dv) {
        if (dv && Sv > T(0)) {
            const T w = (T)wv;
            if (UNIT) {
                for (int k = 0; k < kRB; ++k) acc[k] += w;
            } else {
                // (b / S)^(p-1) = 2^((p-1) log2 b - (p-1) log2 S); b = 0 gives 2^-inf = 0
                const T lS = pm1 * vlog2(Sv);
                const T x = (T)ix, y = (T)iy;
                for (int k = 0; k < kRB; ++k) {
                    const T b = fmax(cone(x, y, r[k], c2), T(0));
                    acc[k] = fma(w, vexp2(fma(pm1, vlog2(b), -lS)), acc[k]);
                }
            }
        }
        ix += qx;
        iy += qy;
        if (ix >= nx) {
            ix -= nx;
            ++iy;
        }
    };
    int c = min(node, last);
    T S0 = S[c];
    double w0 = dJdphi[c];
    uint8_t d0 = design[c];
    for (; node < end; node += 2 * kThreads) {
        c = min(node + kThreads, last);
        const T S1 = S[c];
        const double w1 = dJdphi[c];
        const uint8_t d1 = design[c];
        visit(S0, w0, d0);
        c = min(node + 2 * kThreads, last);
        S0 = S[c];
        w0 = dJdphi[c];
        d0 = design[c];
        if (node + kThreads < end) visit(S1, w1, d1);
    }
    for (int k = 0; k < kRB; ++k) {
        const double v = block_reduce((double)acc[k], OpSum(), red);
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
    // one round of resident blocks (8 blocks of 4 waves per CU): the backward
    // blocks are equal in size, so a second, partial round would only add a tail
    long long want = std::max(1, (2 * kMinBlocks) / P.ngrp);
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

// Optional per-kernel device time of the three pair kernels (process-wide):
// when on, each of their launches carries a start/end event pair bound to the
// dispatch itself.
struct RbfProf {
    struct Rec { int kind; double pairs; hipEvent_t a, b; };
    std::mutex mu;
    bool on = false;
    std::vector<Rec> recs;
    double ms[LLG_RBF_KIND_COUNT] = {0};
    double pairs[LLG_RBF_KIND_COUNT] = {0};
    int64_t n[LLG_RBF_KIND_COUNT] = {0};
};
RbfProf& prof() {
    static RbfProf p;
    return p;
}

// Events for one launch of `kind` covering `pairs` node-RBF pairs (null when off).
void prof_events(int kind, double pairs, hipEvent_t* a, hipEvent_t* b) {
    *a = *b = nullptr;
    RbfProf& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (!P.on) return;
    if (hipEventCreate(a) != hipSuccess) { *a = nullptr; return; }
    if (hipEventCreate(b) != hipSuccess) { (void)hipEventDestroy(*a); *a = *b = nullptr; return; }
    P.recs.push_back({kind, pairs, *a, *b});
}

int prof_drain() {
    RbfProf& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    int rc = LLG_OK;
    for (auto& r : P.recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            rc = llg::set_error(LLG_EHIP, "rbf profile: event timing failed");
        } else {
            P.ms[r.kind] += ms;
            P.pairs[r.kind] += r.pairs;
            P.n[r.kind] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    P.recs.clear();
    return rc;
}

template <typename T, int TPN>
void launch_fwd_passes(const Plan& P, int nx, int nnode, int n, const double* ctr, const double* s, T c2, T p,
                       const uint8_t* design, T* phi, T* S_out, double* work, hipStream_t st) {
    double* part_min = work + 2;
    double* part_max = work + 2 + P.nb;
    const double pairs = (double)nnode * n;
    hipEvent_t a, b;
    prof_events(LLG_RBF_KIND_CONES, pairs, &a, &b);
    hipExtLaunchKernelGGL((k_rbf_cones<T, TPN>), dim3(P.nb), dim3(kThreads), 0, st, a, b, 0, nx, nnode, n, ctr, s, c2,
                          design, phi, part_min);
    k_rbf_finish<<<1, kThreads, 0, st>>>(part_min, P.nb, 0, 0, work);
    prof_events(LLG_RBF_KIND_PNORM, pairs, &a, &b);
    hipExtLaunchKernelGGL((k_rbf_pnorm<T, TPN>), dim3(P.nb), dim3(kThreads), 0, st, a, b, 0, nx, nnode, n, ctr, s, c2,
                          p, design, (const double*)work, phi, S_out, part_max);
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
    hipEvent_t a, b;
    prof_events(LLG_RBF_KIND_VJP, (double)nnode * n, &a, &b);
    if (p == 1.0)
        hipExtLaunchKernelGGL((k_rbf_vjp<T, true>), dim3(P.nchunk, P.ngrp), dim3(kThreads), 0, st, a, b, 0, nx, nnode, n,
                              ctr, s, (T)(c * c), T(0), design, dJdphi, S, work, P.chunk, part);
    else
        hipExtLaunchKernelGGL((k_rbf_vjp<T, false>), dim3(P.nchunk, P.ngrp), dim3(kThreads), 0, st, a, b, 0, nx, nnode,
                              n, ctr, s, (T)(c * c), (T)(p - 1.0), design, dJdphi, S, work, P.chunk, part);
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

int llg_rbf_profile(int enable) {
    if (enable && llg::counter_collection_active())
        return llg::set_error(LLG_ENOTSUP, "event-timed dispatches are not used while hardware counters are collected");
    if (int rc = prof_drain()) return rc;
    RbfProf& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    P.on = enable != 0;
    return LLG_OK;
}

int llg_rbf_profile_read(int32_t kind, double* ms, int64_t* launches, double* pairs, int reset) {
    if (kind < 0 || kind >= LLG_RBF_KIND_COUNT) return llg::set_error(LLG_EINVAL, "rbf profile: bad kind");
    if (int rc = prof_drain()) return rc;
    RbfProf& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (ms) *ms = P.ms[kind];
    if (launches) *launches = P.n[kind];
    if (pairs) *pairs = P.pairs[kind];
    if (reset) {
        P.ms[kind] = 0;
        P.n[kind] = 0;
        P.pairs[kind] = 0;
    }
    return LLG_OK;
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
