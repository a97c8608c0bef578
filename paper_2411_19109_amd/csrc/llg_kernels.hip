// Device kernels of the level-set LLG forward / adjoint path (gfx950).
//
// Data layout (all in HBM, component-major SoA, x fastest):
//   vector fields  v[c*N + (iz*ny + iy)*nx + ix]
//   x-spectrum     S[(c*nrows + row)*Kx + kx], row = iz*ny + iy, kx in [0, Px/2]
//   tensor spectrum nhat[((comp*Kz2 + kz)*Ky2 + ky)*Kx + kx]  (real)
//
// Demag field B_d = -mu0 Ms N * (psi m) is a linear convolution computed with
// zero padding: a real-to-complex FFT along x of each grid row (fused into the
// local kernel that produced the row), one column kernel that transforms along
// y (and z), multiplies by the tensor spectrum and transforms back, and the
// inverse x FFT fused into the next local kernel.  Three real rows are packed
// into complex signals (x,y components of one row; z components of two rows),
// so every row FFT is a complex FFT of length Px.  All FFTs are radix-4/2
// Stockham passes in LDS with precomputed float64-accurate twiddles.
#include <hip/hip_runtime.h>

#include "llg_internal.hpp"

namespace llg {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename C> __device__ __forceinline__ C cmk(decltype(C().x) a, decltype(C().x) b) { C r; r.x = a; r.y = b; return r; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) { return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmk<C>(a.x, -a.y); }
// multiply by +i or -i
template <typename C> __device__ __forceinline__ C cmul_i(C a) { return cmk<C>(-a.y, a.x); }
template <typename C> __device__ __forceinline__ C cmul_mi(C a) { return cmk<C>(a.y, -a.x); }

// ---------------------------------------------------------------------------
// LDS Stockham FFT
// ---------------------------------------------------------------------------
// Signal b occupies buf[(b >> ln0) * s1 + (b & (2^ln0 - 1)) * s0 + e * es], e in [0, L).
struct SigMap {
    int ln0, s1, s0, es;
    __device__ __forceinline__ int off(int b) const { return (b >> ln0) * s1 + (b & ((1 << ln0) - 1)) * s0; }
};

// cos / sin of 2 pi m / 16, m = 0..15 (exact constants)
__device__ constexpr double kC16[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                        0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                        -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                                        0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kS16[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                                        1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                        0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                                        -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

constexpr int bitrev(int i, int lg) {
    int r = 0;
    for (int k = 0; k < lg; ++k) r |= ((i >> k) & 1) << (lg - 1 - k);
    return r;
}
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
__device__ __forceinline__ int ilog2_rt(int v) { return 31 - __clz(v); }

// In-register DFT of size R (power of two <= 16): radix-2 decimation in time
// with constant twiddles; forward sign -1, inverse +1, unnormalised.
template <typename C, bool INV, int R>
__device__ __forceinline__ void dft_small(C* v) {
    using T = decltype(C().x);
    constexpr int LG = ilog2(R);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int j = bitrev(i, LG);
        if (j > i) {
            C t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const C u = v[i + k];
                C t = v[i + k + len / 2];
                const int m = k * (16 / len);  // exp(-+2 pi i k / len) = entry m of the 16-point table
                if (m == 0) {
                } else if (m == 4) {
                    t = INV ? cmul_i(t) : cmul_mi(t);
                } else {
                    const C w = cmk<C>((T)kC16[m], INV ? (T)kS16[m] : -(T)kS16[m]);
                    t = cmul(t, w);
                }
                v[i + k] = cadd(u, t);
                v[i + k + len / 2] = csub(u, t);
            }
        }
    }
}

// One Stockham pass of radix R over nsig signals of length L = 2^lL (in place
// via registers).  Requires nsig * L <= MAXREG * blockDim.x.
template <typename C, bool INV, int R, int MAXREG>
__device__ __forceinline__ void fft_pass(C* buf, const SigMap sm, int lL, int lNs, int nsig, const C* __restrict__ tw) {
    constexpr int IPT = MAXREG / R;
    constexpr int LR = ilog2(R);
    const int lnbf = lL - LR;
    const int nbf = 1 << lnbf;
    const int total = nsig << lnbf;
    C v[IPT][R];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int it = threadIdx.x + q * blockDim.x;
        if (it < total) {
            const int b = it >> lnbf, j = it & (nbf - 1);
            const C* s = buf + sm.off(b);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = s[(j + (r << lnbf)) * sm.es];
        }
    }
    __syncthreads();
    const int lstride = lL - lNs - LR;  // twiddle index step L / (Ns R)
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int it = threadIdx.x + q * blockDim.x;
        if (it < total) {
            const int b = it >> lnbf, j = it & (nbf - 1);
            const int jm = j & ((1 << lNs) - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C w = tw[(r * jm) << lstride];
                if (INV) w = cconj(w);
                v[q][r] = cmul(v[q][r], w);
            }
            dft_small<C, INV, R>(v[q]);
            C* d = buf + sm.off(b);
            const int base = ((j - jm) << LR) + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) d[(base + (r << lNs)) * sm.es] = v[q][r];
        }
    }
    __syncthreads();
}

// Full FFT of length L (power of two) of nsig signals; tw = exp(-2 pi i k / L).
// Radix-16 passes while at least 16 points remain per sub-transform, then one
// pass of the remaining radix (8, 4 or 2).
template <typename C, bool INV, int MAXREG>
__device__ void fft_lds(C* buf, const SigMap sm, int L, int nsig, const C* __restrict__ tw) {
    int lL = 0;
    while ((1 << lL) < L) ++lL;
    int lNs = 0;
    while (lNs < lL) {
        const int rem = lL - lNs;
        if (rem >= 4) {
            fft_pass<C, INV, 16, MAXREG>(buf, sm, lL, lNs, nsig, tw);
            lNs += 4;
        } else if (rem == 3) {
            fft_pass<C, INV, 8, MAXREG>(buf, sm, lL, lNs, nsig, tw);
            lNs += 3;
        } else if (rem == 2) {
            fft_pass<C, INV, 4, MAXREG>(buf, sm, lL, lNs, nsig, tw);
            lNs += 2;
        } else {
            fft_pass<C, INV, 2, MAXREG>(buf, sm, lL, lNs, nsig, tw);
            lNs += 1;
        }
    }
}

template <typename T> struct MaxReg;
template <> struct MaxReg<float> { static constexpr int v = 32; };
template <> struct MaxReg<double> { static constexpr int v = 16; };

// ---------------------------------------------------------------------------
// node-local physics helpers
// ---------------------------------------------------------------------------
template <typename T> struct V3 { T x, y, z; };
template <typename T> __device__ __forceinline__ V3<T> v3(T a, T b, T c) { return V3<T>{a, b, c}; }
template <typename T> __device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
template <typename T> __device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
template <typename T> __device__ __forceinline__ V3<T> operator*(T s, V3<T> a) { return v3(s * a.x, s * a.y, s * a.z); }
template <typename T> __device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <typename T> __device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

template <typename T> __device__ __forceinline__ V3<T> ld3(const T* __restrict__ v, int N, int i) {
    return v3(v[i], v[N + i], v[2 * N + i]);
}
template <typename T> __device__ __forceinline__ void st3(T* __restrict__ v, int N, int i, V3<T> a) {
    v[i] = a.x;
    v[N + i] = a.y;
    v[2 * N + i] = a.z;
}

// Damping of node (ix, iy, iz): linear ramp over ramp_cells nodes from each ramped face.
template <typename T> __device__ __forceinline__ T node_alpha(const KParams<T>& p, int ix, int iy, int iz) {
    if (p.ramp_cells <= 0 || p.ramp_faces == 0) return p.alpha0;
    int d = 0x3fffffff;
    if (p.ramp_faces & 1) d = min(d, ix);
    if (p.ramp_faces & 2) d = min(d, p.nx - 1 - ix);
    if (p.ramp_faces & 4) d = min(d, iy);
    if (p.ramp_faces & 8) d = min(d, p.ny - 1 - iy);
    if (p.ramp_faces & 16) d = min(d, iz);
    if (p.ramp_faces & 32) d = min(d, p.nz - 1 - iz);
    const int w = p.ramp_cells - d;
    if (w <= 0) return p.alpha0;
    return p.alpha0 + (p.alpha_max - p.alpha0) * ((T)w / (T)p.ramp_cells);
}

__device__ __forceinline__ double drive_value(double f1, double f2, double tsw, double t) {
    const double twopi = 6.283185307179586476925286766559;
    double ph = (tsw > 0.0 && t >= tsw) ? twopi * (f1 * tsw + f2 * (t - tsw)) : twopi * f1 * t;
    return sin(ph);
}

// Exchange field at node i (flat), neighbours along each axis with free ends:
// B = sum_j exw_d psi_j/(psi_i+psi_j) (m_j - m_i).
template <typename T>
__device__ __forceinline__ V3<T> exchange_field(const KParams<T>& p, const T* __restrict__ y, const T* __restrict__ psi,
                                                int i, int ix, int iy, int iz, V3<T> mi, T pi) {
    V3<T> B = v3<T>(0, 0, 0);
    const int N = p.N;
    auto add = [&](int j, T w) {
        const T pj = psi[j];
        const T s = pi + pj;
        if (s != (T)0) {
            const T c = w * pj / s;
            B = B + c * (ld3(y, N, j) - mi);
        }
    };
    if (ix > 0) add(i - 1, p.exw[0]);
    if (ix < p.nx - 1) add(i + 1, p.exw[0]);
    if (iy > 0) add(i - p.nx, p.exw[1]);
    if (iy < p.ny - 1) add(i + p.nx, p.exw[1]);
    if (iz > 0) add(i - p.nx * p.ny, p.exw[2]);
    if (iz < p.nz - 1) add(i + p.nx * p.ny, p.exw[2]);
    return B;
}

// ---------------------------------------------------------------------------
// spectrum row packing: rows r0, r1 -> three complex signals of length Px
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void unpack_rows_to_lds(const KParams<T>& p, const cplx<T>* __restrict__ S, int r0, bool v1,
                                                   cplx<T>* Z) {
    using C = cplx<T>;
    const int Px = p.Px, Kx = p.Kx;
    const size_t cs = (size_t)p.nrows * Kx;
    for (int k = threadIdx.x; k < Px; k += blockDim.x) {
        const bool cj = k > Px / 2;
        const int kk = cj ? Px - k : k;
        const C* s0 = S + (size_t)r0 * Kx + kk;
        C ax = s0[0], ay = s0[cs], az = s0[2 * cs];
        C bx = cmk<C>(0, 0), by = bx, bz = bx;
        if (v1) {
            bx = s0[Kx];
            by = s0[Kx + cs];
            bz = s0[Kx + 2 * cs];
        }
        if (cj) {
            ax = cconj(ax); ay = cconj(ay); az = cconj(az);
            bx = cconj(bx); by = cconj(by); bz = cconj(bz);
        }
        Z[k] = cadd(ax, cmul_i(ay));
        Z[Px + k] = cadd(bx, cmul_i(by));
        Z[2 * Px + k] = cadd(az, cmul_i(bz));
    }
}

template <typename T>
__device__ __forceinline__ void pack_lds_to_rows(const KParams<T>& p, cplx<T>* __restrict__ S, int r0, bool v1,
                                                 const cplx<T>* Z) {
    using C = cplx<T>;
    const int Px = p.Px, Kx = p.Kx;
    const size_t cs = (size_t)p.nrows * Kx;
    const T h = (T)0.5;
    for (int k = threadIdx.x; k < Kx; k += blockDim.x) {
        const int kn = (Px - k) & (Px - 1);
        C out[6];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const C a = Z[s * Px + k];
            const C b = cconj(Z[s * Px + kn]);
            const C sum = cadd(a, b), dif = csub(a, b);
            out[2 * s] = cmk<C>(h * sum.x, h * sum.y);       // spectrum of the real part
            out[2 * s + 1] = cmk<C>(h * dif.y, -h * dif.x);  // spectrum of the imaginary part
        }
        C* d = S + (size_t)r0 * Kx + k;
        d[0] = out[0];
        d[cs] = out[1];
        d[2 * cs] = out[4];
        if (v1) {
            d[Kx] = out[2];
            d[Kx + cs] = out[3];
            d[Kx + 2 * cs] = out[5];
        }
    }
}

// ---------------------------------------------------------------------------
// shared-memory layout of the local (row-pair) kernels
//   Z  [3 * Px] complex  three packed row signals (demag only)
//   Tw [Px]     complex  x twiddles (demag only)
//   R  [4][NV][nx] real  rows r0-1 .. r0+2 of NV staged node values
// Staging the two own rows and their two y-neighbour rows lets every x and y
// neighbour of the stencil come from LDS; the loads are issued together with
// the spectrum loads, before the first FFT pass.
// ---------------------------------------------------------------------------
template <typename T>
struct LocalSmem {
    cplx<T>* Z;
    cplx<T>* Tw;
    T* R;
};

template <typename T>
__device__ __forceinline__ LocalSmem<T> local_smem(unsigned char* raw, int Px, bool demag) {
    LocalSmem<T> L;
    L.Z = reinterpret_cast<cplx<T>*>(raw);
    L.Tw = L.Z + (demag ? 3 * Px : 0);
    L.R = reinterpret_cast<T*>(L.Tw + (demag ? Px : 0));
    return L;
}

// Stage rows r0-1 .. r0+2 of NV arrays src[v] (component-major vectors use
// stride N) into R; rows outside the grid are left unset (never read).
template <typename T, int NV>
__device__ __forceinline__ void stage_rows(const KParams<T>& p, int r0, const T* const (&src)[NV], const int (&comp)[NV],
                                           T* R) {
    const int nx = p.nx;
    for (int e = threadIdx.x; e < 4 * nx; e += blockDim.x) {
        const int q = e / nx, x = e - q * nx;
        const int r = r0 - 1 + q;
        if (r < 0 || r >= p.nrows) continue;
        const int i = r * nx + x;
#pragma unroll
        for (int v = 0; v < NV; ++v) R[(q * NV + v) * nx + x] = src[v][comp[v] * p.N + i];
    }
}

// ---------------------------------------------------------------------------
// forward local kernel: inverse x-FFT (demag) + local field + LL RHS + RK4
// stage update + forward x-FFT of the next stage's magnetisation
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) k_stage_fwd(const KParams<T> p, const StageFwdArgs<T> a,
                                                   const cplx<T>* __restrict__ twx) {
    using C = cplx<T>;
    constexpr int NV = 4;  // m_x, m_y, m_z, psi
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][512 / 64];
    const int Px = p.Px, nx = p.nx, N = p.N;
    const bool demag_in = a.do_inv != 0, demag_any = (a.do_inv | a.do_fwd) != 0;
    const LocalSmem<T> L = local_smem<T>(smem_raw, Px, demag_any);
    C* Z = L.Z;
    T* R = L.R;
    const int r0 = 2 * blockIdx.x;
    const bool v1 = r0 + 1 < p.nrows;
    constexpr int MR = MaxReg<T>::v;
    const SigMap sm{0, Px, 0, 1};

    {
        const T* const src[NV] = {a.ys, a.ys, a.ys, a.psi};
        const int comp[NV] = {0, 1, 2, 0};
        stage_rows<T, NV>(p, r0, src, comp, R);
    }
    if (demag_any)
        for (int k = threadIdx.x; k < Px; k += blockDim.x) L.Tw[k] = twx[k];
    if (demag_in) unpack_rows_to_lds(p, a.S, r0, v1, Z);
    __syncthreads();
    if (demag_in) fft_lds<C, true, MR>(Z, sm, Px, 3, L.Tw);

    const T drv = (T)drive_value(p.f1, p.f2, p.t_switch, a.t);
    const T dt = p.dt;
    double s1 = 0.0, s2 = 0.0;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        T out[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int r = r0 + rr;
            if (rr == 1 && !v1) break;
            const int q = rr + 1;
            const int iy = r % p.ny, iz = r / p.ny;
            const int i = r * nx + x;
            auto RM = [&](int qq, int xx) {
                return v3<T>(R[(qq * NV + 0) * nx + xx], R[(qq * NV + 1) * nx + xx], R[(qq * NV + 2) * nx + xx]);
            };
            auto RP = [&](int qq, int xx) { return R[(qq * NV + 3) * nx + xx]; };
            const V3<T> m = RM(q, x);
            const T pi = RP(q, x);
            V3<T> B = v3<T>(0, 0, 0);
            if (demag_in) {
                const C z01 = Z[rr * Px + x];
                const C z2 = Z[2 * Px + x];
                B = v3<T>(z01.x, z01.y, rr == 0 ? z2.x : z2.y);
            }
            if (p.terms & 1) {
                // exchange: sum_j exw_d psi_j/(psi_i+psi_j) (m_j - m_i), free ends
                V3<T> Be = v3<T>(0, 0, 0);
                auto add = [&](V3<T> mj, T pj, T w) {
                    const T s = pi + pj;
                    if (s != (T)0) Be = Be + (w * pj / s) * (mj - m);
                };
                if (x > 0) add(RM(q, x - 1), RP(q, x - 1), p.exw[0]);
                if (x < nx - 1) add(RM(q, x + 1), RP(q, x + 1), p.exw[0]);
                if (iy > 0) add(RM(q - 1, x), RP(q - 1, x), p.exw[1]);
                if (iy < p.ny - 1) add(RM(q + 1, x), RP(q + 1, x), p.exw[1]);
                if (iz > 0) add(ld3(a.ys, N, i - nx * p.ny), a.psi[i - nx * p.ny], p.exw[2]);
                if (iz < p.nz - 1) add(ld3(a.ys, N, i + nx * p.ny), a.psi[i + nx * p.ny], p.exw[2]);
                B = B + Be;
            }
            if (p.terms & 4) {
                B = B + v3<T>(p.B0[0], p.B0[1], p.B0[2]);
                if (a.antenna && a.antenna[i]) B = B + drv * v3<T>(p.brf[0], p.brf[1], p.brf[2]);
            }
            if (p.terms & 8) {
                const V3<T> u = v3<T>(p.u[0], p.u[1], p.u[2]);
                B = B + (p.anis * dot(m, u)) * u;
            }
            V3<T> f = v3<T>(0, 0, 0);
            if (pi != (T)0) {
                const T al = node_alpha(p, x, iy, iz);
                const T gp = p.gamma / ((T)1 + al * al);
                const V3<T> c = cross(m, B);
                f = (-gp) * (c + al * cross(m, c));
            }
            if (a.ys_store) st3(a.ys_store, N, i, m);
            if (a.Bs_store) st3(a.Bs_store, N, i, B);
            V3<T> yn;
            if (a.stage == -3) {
                yn = m;  // prologue: spectrum of psi * m only
            } else if (a.stage < 0) {
                yn = f;  // field evaluation: rhs out
            } else if (a.stage == 0) {
                st3(a.acc, N, i, m + (dt / (T)6) * f);
                yn = m + (dt / (T)2) * f;
            } else if (a.stage == 1) {
                st3(a.acc, N, i, ld3(a.acc, N, i) + (dt / (T)3) * f);
                yn = ld3(a.mn, N, i) + (dt / (T)2) * f;
            } else if (a.stage == 2) {
                st3(a.acc, N, i, ld3(a.acc, N, i) + (dt / (T)3) * f);
                yn = ld3(a.mn, N, i) + dt * f;
            } else {
                yn = ld3(a.acc, N, i) + (dt / (T)6) * f;
            }
            if (a.ynext) st3(a.ynext, N, i, yn);
            if (a.port_part) {
                const double my2 = (double)yn.y * (double)yn.y;
                if (a.port1[i]) s1 += my2;
                if (a.port2[i]) s2 += my2;
            }
            out[rr][0] = pi * yn.x;
            out[rr][1] = pi * yn.y;
            out[rr][2] = pi * yn.z;
        }
        if (a.do_fwd) {
            Z[x] = cmk<C>(out[0][0], out[0][1]);
            Z[Px + x] = cmk<C>(out[1][0], out[1][1]);
            Z[2 * Px + x] = cmk<C>(out[0][2], out[1][2]);
        }
    }
    if (a.port_part) {
        // deterministic block reduction: wave shuffles, then a fixed-order sum of the waves
        for (int o = 32; o > 0; o >>= 1) {
            s1 += __shfl_down(s1, o, 64);
            s2 += __shfl_down(s2, o, 64);
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][w] = s1;
            red[1][w] = s2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double t1 = 0.0, t2 = 0.0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
                t1 += red[0][k];
                t2 += red[1][k];
            }
            a.port_part[2 * blockIdx.x] += t1;
            a.port_part[2 * blockIdx.x + 1] += t2;
        }
    }
    if (a.do_fwd) {
        for (int x = nx + threadIdx.x; x < Px; x += blockDim.x) {
            Z[x] = cmk<C>(0, 0);
            Z[Px + x] = cmk<C>(0, 0);
            Z[2 * Px + x] = cmk<C>(0, 0);
        }
        __syncthreads();
        fft_lds<C, false, MR>(Z, sm, Px, 3, L.Tw);
        pack_lds_to_rows(p, a.S, r0, v1, Z);
    }
}

// ---------------------------------------------------------------------------
// backward local kernel: transpose of one RK stage (see the adjoint notes in
// the runtime), accumulation of dJ/dpsi, and preparation of the next stage's
// field adjoint u and its x-spectrum
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ V3<T> field_adjoint(const KParams<T>& p, V3<T> ell, V3<T> m, int ix, int iy, int iz, T psi_i) {
    if (psi_i == (T)0) return v3<T>(0, 0, 0);
    const T al = node_alpha(p, ix, iy, iz);
    const T gp = p.gamma / ((T)1 + al * al);
    const V3<T> w = cross(ell, m);
    return (-gp) * (w + al * cross(w, m));
}

template <typename T>
__global__ void __launch_bounds__(512) k_stage_bwd(const KParams<T> p, const StageBwdArgs<T> a,
                                                   const cplx<T>* __restrict__ twx) {
    using C = cplx<T>;
    constexpr int NV = 4;  // u_x, u_y, u_z, psi
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int Px = p.Px, nx = p.nx, N = p.N;
    const bool seed = a.stage < 0;
    const bool demag_in = a.do_inv && !seed, demag_any = (a.do_inv | a.do_fwd) != 0;
    const LocalSmem<T> L = local_smem<T>(smem_raw, Px, demag_any);
    C* Z = L.Z;
    T* R = L.R;
    const int r0 = 2 * blockIdx.x;
    const bool v1 = r0 + 1 < p.nrows;
    constexpr int MR = MaxReg<T>::v;
    const SigMap sm{0, Px, 0, 1};

    if (!seed && (p.terms & 1)) {
        const T* const src[NV] = {a.u_cur, a.u_cur, a.u_cur, a.psi};
        const int comp[NV] = {0, 1, 2, 0};
        stage_rows<T, NV>(p, r0, src, comp, R);
    }
    if (demag_any)
        for (int k = threadIdx.x; k < Px; k += blockDim.x) L.Tw[k] = twx[k];
    if (demag_in) unpack_rows_to_lds(p, a.S, r0, v1, Z);
    __syncthreads();
    if (demag_in) fft_lds<C, true, MR>(Z, sm, Px, 3, L.Tw);

    const T dt = p.dt;
    // l_{s-1} = cl lambda' + cm mu_s (0-based stages): RK4 weights b = (1,2,2,1)/6 and nodes c = (0,1/2,1/2,1)
    const T cl = (a.stage == 1) ? dt / (T)6 : dt / (T)3;
    const T cm = (a.stage == 3) ? dt : dt / (T)2;

    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        T out[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int r = r0 + rr;
            if (rr == 1 && !v1) break;
            const int q = rr + 1;
            const int iy = r % p.ny, iz = r / p.ny;
            const int i = r * nx + x;
            const T pi = a.psi[i];
            V3<T> un = v3<T>(0, 0, 0);
            if (seed) {
                const V3<T> lam = ld3(a.lamp, N, i);
                const V3<T> ell = (dt / (T)6) * lam;
                st3(a.ell, N, i, ell);
                un = field_adjoint(p, ell, ld3(a.y_prev, N, i), x, iy, iz, pi);
                st3(a.u_next, N, i, un);
            } else {
                const V3<T> m = ld3(a.ys, N, i);
                const V3<T> B = ld3(a.Bs, N, i);
                const V3<T> v = ld3(a.ell, N, i);
                const V3<T> uk = ld3(a.u_cur, N, i);
                V3<T> mu = v3<T>(0, 0, 0);
                if (pi != (T)0) {
                    const T al = node_alpha(p, x, iy, iz);
                    const T gp = p.gamma / ((T)1 + al * al);
                    const V3<T> w = cross(v, m);
                    const V3<T> c = cross(m, B);
                    mu = (-gp) * (cross(B, v) + al * cross(c, v) + al * cross(B, w));
                }
                double g = 0.0;
                if (p.terms & 1) {
                    // exchange transpose and psi-gradient over the neighbours j of i:
                    //   mu_i += exw psi_i/s u_j - exw psi_j/s u_i
                    //   g_i  -= exw psi_j/s^2 (u_i + u_j).(m_j - m_i),   s = psi_i + psi_j
                    auto RU = [&](int qq, int xx) {
                        return v3<T>(R[(qq * NV + 0) * nx + xx], R[(qq * NV + 1) * nx + xx], R[(qq * NV + 2) * nx + xx]);
                    };
                    auto RP = [&](int qq, int xx) { return R[(qq * NV + 3) * nx + xx]; };
                    auto nb = [&](V3<T> uj, T pj, int j, T w) {
                        const T s = pi + pj;
                        if (s != (T)0) {
                            const V3<T> mj = ld3(a.ys, N, j);
                            const T is = (T)1 / s;
                            mu = mu + (w * pi * is) * uj - (w * pj * is) * uk;
                            g -= (double)(w * pj * is * is) * (double)dot(uk + uj, mj - m);
                        }
                    };
                    if (x > 0) nb(RU(q, x - 1), RP(q, x - 1), i - 1, p.exw[0]);
                    if (x < nx - 1) nb(RU(q, x + 1), RP(q, x + 1), i + 1, p.exw[0]);
                    if (iy > 0) nb(RU(q - 1, x), RP(q - 1, x), i - nx, p.exw[1]);
                    if (iy < p.ny - 1) nb(RU(q + 1, x), RP(q + 1, x), i + nx, p.exw[1]);
                    if (iz > 0) nb(ld3(a.u_cur, N, i - nx * p.ny), a.psi[i - nx * p.ny], i - nx * p.ny, p.exw[2]);
                    if (iz < p.nz - 1) nb(ld3(a.u_cur, N, i + nx * p.ny), a.psi[i + nx * p.ny], i + nx * p.ny, p.exw[2]);
                }
                if (demag_in) {
                    const C z01 = Z[rr * Px + x];
                    const C z2 = Z[2 * Px + x];
                    const V3<T> cu = v3<T>(z01.x, z01.y, rr == 0 ? z2.x : z2.y);
                    mu = mu + pi * cu;
                    g += (double)dot(m, cu);
                }
                if (p.terms & 8) {
                    const V3<T> ua = v3<T>(p.u[0], p.u[1], p.u[2]);
                    mu = mu + (p.anis * dot(uk, ua)) * ua;
                }
                a.gpsi[i] += g;
                const V3<T> lsum = (a.stage == 3 ? ld3(a.lamp, N, i) : ld3(a.lacc_in, N, i)) + mu;
                if (a.stage > 0) {
                    st3(a.lacc_out, N, i, lsum);
                    const V3<T> ell = cl * ld3(a.lamp, N, i) + cm * mu;
                    st3(a.ell, N, i, ell);
                    un = field_adjoint(p, ell, ld3(a.y_prev, N, i), x, iy, iz, pi);
                    st3(a.u_next, N, i, un);
                } else {
                    V3<T> lam = lsum;
                    if (a.port1) {
                        // running-cost source dJ/dm_n of the port objective (y component)
                        const T src = (a.port1[i] ? a.src1 : (T)0) - (a.port2[i] ? a.src2 : (T)0);
                        lam.y = lam.y + src * m.y;
                    }
                    st3(a.lacc_out, N, i, lam);
                    if (a.y_prev) {
                        const V3<T> ell = (dt / (T)6) * lam;
                        st3(a.ell, N, i, ell);
                        un = field_adjoint(p, ell, ld3(a.y_prev, N, i), x, iy, iz, pi);
                        st3(a.u_next, N, i, un);
                    }
                }
            }
            out[rr][0] = un.x;
            out[rr][1] = un.y;
            out[rr][2] = un.z;
        }
        if (a.do_fwd) {
            Z[x] = cmk<C>(out[0][0], out[0][1]);
            Z[Px + x] = cmk<C>(out[1][0], out[1][1]);
            Z[2 * Px + x] = cmk<C>(out[0][2], out[1][2]);
        }
    }
    if (a.do_fwd) {
        for (int x = nx + threadIdx.x; x < Px; x += blockDim.x) {
            Z[x] = cmk<C>(0, 0);
            Z[Px + x] = cmk<C>(0, 0);
            Z[2 * Px + x] = cmk<C>(0, 0);
        }
        __syncthreads();
        fft_lds<C, false, MR>(Z, sm, Px, 3, L.Tw);
        pack_lds_to_rows(p, a.S, r0, v1, Z);
    }
}

// ---------------------------------------------------------------------------
// column kernel: y (and z) transforms + tensor-spectrum multiply, in place
// shared memory: Z [c][z < nz][y < Py][tk] complex, Tw [Py] complex,
//                Nt [comp][kz <= Pz/2][ky <= Py/2][tk] real
// ---------------------------------------------------------------------------
template <typename T, int NZ>
__global__ void __launch_bounds__(512) k_col_conv(const KParams<T> p, cplx<T>* __restrict__ S,
                                                  const T* __restrict__ nhat, const cplx<T>* __restrict__ twy,
                                                  const cplx<T>* __restrict__ twz, int TK) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int MR = MaxReg<T>::v;
    const int Kx = p.Kx, Py = p.Py, Pz = p.Pz, ny = p.ny, nz = p.nz;
    const int plane = Py * TK;
    C* Z = reinterpret_cast<C*>(smem_raw);
    C* Tw = Z + 3 * nz * plane;
    T* Nt = reinterpret_cast<T*>(Tw + Py);
    const int k0 = blockIdx.x * TK;
    const size_t cs = (size_t)p.nrows * Kx;
    // load the columns (zero-padded in y), the twiddles and this tile of the tensor spectrum
    const int nload = 3 * nz * Py * TK;
    for (int e = threadIdx.x; e < nload; e += blockDim.x) {
        const int tk = e % TK;
        int t = e / TK;
        const int y = t % Py;
        t /= Py;
        const int z = t % nz, c = t / nz;
        C v = cmk<C>(0, 0);
        if (y < ny && k0 + tk < Kx) v = S[c * cs + (size_t)(z * ny + y) * Kx + k0 + tk];
        Z[e] = v;
    }
    for (int k = threadIdx.x; k < Py; k += blockDim.x) Tw[k] = twy[k];
    const int ntile = p.ncomp * p.Kz2 * p.Ky2 * TK;
    for (int e = threadIdx.x; e < ntile; e += blockDim.x) {
        const int tk = e % TK, row = e / TK;  // row = (comp * Kz2 + kz) * Ky2 + ky
        Nt[e] = (k0 + tk < Kx) ? nhat[(size_t)row * Kx + k0 + tk] : (T)0;
    }
    __syncthreads();
    const SigMap smy{ilog2_rt(TK), plane, 1, TK};
    if (Py > 1) fft_lds<C, false, MR>(Z, smy, Py, 3 * nz * TK, Tw);

    // per (ky, tk): z transform in registers, tensor multiply, inverse z transform
    const int npair = Py * TK;
    const int cstr = p.Kz2 * p.Ky2 * TK;
    for (int e = threadIdx.x; e < npair; e += blockDim.x) {
        const int tk = e % TK, ky = e / TK;
        const int kx = k0 + tk;
        if (kx >= Kx) continue;
        C X[3][NZ];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                X[c][z] = z < nz ? Z[(c * nz + z) * plane + ky * TK + tk] : cmk<C>(0, 0);
        const bool fy = ky > Py / 2;
        const int kyr = fy ? Py - ky : ky;
        C Y[3][NZ];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int z = 0; z < NZ; ++z) Y[c][z] = cmk<C>(0, 0);
        for (int kz = 0; kz < Pz; ++kz) {
            // forward z DFT of the nz nonzero planes
            C h[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                C s = X[c][0];
#pragma unroll
                for (int z = 1; z < NZ; ++z)
                    if (z < nz) s = cadd(s, cmul(X[c][z], twz[(kz * z) & (Pz - 1)]));
                h[c] = s;
            }
            const bool fz = kz > Pz / 2;
            const int kzr = fz ? Pz - kz : kz;
            const int base = (kzr * p.Ky2 + kyr) * TK + tk;
            const T nxx = Nt[base], nyy = Nt[cstr + base], nzz = Nt[2 * cstr + base];
            const T nxy = fy ? -Nt[3 * cstr + base] : Nt[3 * cstr + base];
            T nxz = 0, nyz = 0;
            if (p.ncomp == 6) {
                nxz = fz ? -Nt[4 * cstr + base] : Nt[4 * cstr + base];
                nyz = Nt[5 * cstr + base];
                if (fy != fz) nyz = -nyz;
            }
            const C hx = cmk<C>(nxx * h[0].x + nxy * h[1].x + nxz * h[2].x, nxx * h[0].y + nxy * h[1].y + nxz * h[2].y);
            const C hy = cmk<C>(nxy * h[0].x + nyy * h[1].x + nyz * h[2].x, nxy * h[0].y + nyy * h[1].y + nyz * h[2].y);
            const C hz = cmk<C>(nxz * h[0].x + nyz * h[1].x + nzz * h[2].x, nxz * h[0].y + nyz * h[1].y + nzz * h[2].y);
            // inverse z DFT, only the nz planes that are kept
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                if (z >= nz) break;
                const C w = cconj(twz[(kz * z) & (Pz - 1)]);
                Y[0][z] = cadd(Y[0][z], cmul(hx, w));
                Y[1][z] = cadd(Y[1][z], cmul(hy, w));
                Y[2][z] = cadd(Y[2][z], cmul(hz, w));
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                if (z < nz) Z[(c * nz + z) * plane + ky * TK + tk] = Y[c][z];
    }
    __syncthreads();
    if (Py > 1) fft_lds<C, true, MR>(Z, smy, Py, 3 * nz * TK, Tw);
    const int nstore = 3 * nz * ny * TK;
    for (int e = threadIdx.x; e < nstore; e += blockDim.x) {
        const int tk = e % TK;
        int t = e / TK;
        const int y = t % ny;
        t /= ny;
        const int z = t % nz, c = t / nz;
        if (k0 + tk < Kx) S[c * cs + (size_t)(z * ny + y) * Kx + k0 + tk] = Z[((c * nz + z) * Py + y) * TK + tk];
    }
}

// ---------------------------------------------------------------------------
// level set, objectives, small helpers
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_levelset(const KParams<T> p, const T* __restrict__ phi, const T* __restrict__ psi_fixed,
                           const uint8_t* __restrict__ design, T a, int extrude, T* __restrict__ psi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const int j = extrude ? i % (p.nx * p.ny) : i;
    const T fixed = psi_fixed ? psi_fixed[i] : (T)0;
    psi[i] = (design && design[i]) ? (T)1 / ((T)1 + exp(-a * phi[j])) : fixed;
}

template <typename T>
__global__ void k_levelset_vjp(const KParams<T> p, const T* __restrict__ phi, const double* __restrict__ g,
                               const uint8_t* __restrict__ design, double a, int extrude, double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int M = extrude ? p.nx * p.ny : p.N;
    if (j >= M) return;
    const int nl = extrude ? p.nz : 1;
    const double H = 1.0 / (1.0 + exp(-a * (double)phi[j]));
    const double hp = a * H * (1.0 - H);
    double s = 0.0;
    for (int l = 0; l < nl; ++l) {
        const int i = j + l * M;
        if (design && design[i]) s += hp * g[i];
    }
    out[j] = s;
}

// Energy terms, dJ/dm and explicit dJ/dpsi of the energy + area objective,
// with per-block partial sums (ex, d, Z, an, psi) in fixed order.
template <typename T>
__global__ void __launch_bounds__(512) k_energy(const KParams<T> p, double t, const T* __restrict__ psi,
                                                const T* __restrict__ m, const cplx<T>* __restrict__ S,
                                                const cplx<T>* __restrict__ twx, const uint8_t* __restrict__ antenna,
                                                double scale, T* __restrict__ dJdm, double* __restrict__ dJdpsi,
                                                double* __restrict__ part) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* Z = reinterpret_cast<C*>(smem_raw);
    __shared__ double red[5][512 / 64];
    const int r0 = 2 * blockIdx.x;
    const bool v1 = r0 + 1 < p.nrows;
    const int Px = p.Px;
    constexpr int MR = MaxReg<T>::v;
    const bool demag = (p.terms & 2) != 0;
    if (demag) {
        unpack_rows_to_lds(p, S, r0, v1, Z);
        __syncthreads();
        fft_lds<C, true, MR>(Z, SigMap{0, Px, 0, 1}, Px, 3, twx);
    }
    const T drv = (T)drive_value(p.f1, p.f2, p.t_switch, t);
    const int N = p.N, nx = p.nx;
    double e[5] = {0, 0, 0, 0, 0};
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        for (int rr = 0; rr < 2; ++rr) {
            const int r = r0 + rr;
            if (rr == 1 && !v1) break;
            const int iy = r % p.ny, iz = r / p.ny;
            const int i = r * nx + x;
            const V3<T> mi = ld3(m, N, i);
            const T pi = psi[i];
            V3<T> Bd = v3<T>(0, 0, 0), Bex = v3<T>(0, 0, 0);
            if (demag) {
                const C z01 = Z[rr * Px + x];
                const C z2 = Z[2 * Px + x];
                Bd = v3<T>(z01.x, z01.y, rr == 0 ? z2.x : z2.y);
            }
            double gp = 0.0;
            if (p.terms & 1) {
                Bex = exchange_field(p, m, psi, i, x, iy, iz, mi, pi);
                // E_ex / (Ms V) = sum over edges of exw/2 psi_i psi_j / s |dm|^2 (each edge once, from its
                // lower node); d(E_ex/(Ms V))/dpsi_i = sum over neighbours of exw/2 psi_j^2 / s^2 |dm|^2
                auto edge = [&](int j, T w, bool fwd) {
                    const T pj = psi[j];
                    const T s = pi + pj;
                    if (s != (T)0) {
                        const V3<T> d = ld3(m, N, j) - mi;
                        const double d2 = (double)dot(d, d);
                        if (fwd) e[0] += 0.5 * (double)(w * pi * pj / s) * d2;
                        gp += 0.5 * (double)(w * pj * pj / (s * s)) * d2;
                    }
                };
                if (x > 0) edge(i - 1, p.exw[0], false);
                if (x < nx - 1) edge(i + 1, p.exw[0], true);
                if (iy > 0) edge(i - nx, p.exw[1], false);
                if (iy < p.ny - 1) edge(i + nx, p.exw[1], true);
                if (iz > 0) edge(i - nx * p.ny, p.exw[2], false);
                if (iz < p.nz - 1) edge(i + nx * p.ny, p.exw[2], true);
            }
            // energies in units of Ms * V (the host multiplies by Ms V)
            e[1] += -0.5 * (double)pi * (double)dot(mi, Bd);
            if (p.terms & 4) {
                V3<T> Bz = v3<T>(p.B0[0], p.B0[1], p.B0[2]);
                if (antenna && antenna[i]) Bz = Bz + drv * v3<T>(p.brf[0], p.brf[1], p.brf[2]);
                e[2] += -(double)pi * (double)dot(mi, Bz);
            }
            if (p.terms & 8) {
                const V3<T> u = v3<T>(p.u[0], p.u[1], p.u[2]);
                const double mu = (double)dot(mi, u);
                e[3] += -0.5 * (double)p.anis * (double)pi * mu * mu;
            }
            e[4] += (double)pi;
            // dJ/dm = -(Ms V / E_ref) psi (B_ex + B_d); explicit dJ/dpsi without the area term
            const V3<T> Bt = Bex + Bd;
            const T sc = (T)(-scale) * pi;
            if (dJdm) st3(dJdm, N, i, sc * Bt);
            if (dJdpsi) dJdpsi[i] = scale * (gp - (double)dot(mi, Bd));
        }
    }
    for (int q = 0; q < 5; ++q)
        for (int o = 32; o > 0; o >>= 1) e[q] += __shfl_down(e[q], o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 5; ++q) red[q][w] = e[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 5; ++q) {
            double s = 0.0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[q][k];
            part[5 * blockIdx.x + q] = s;
        }
    }
}

// Single-block fixed-order reduction of the energy partials.
// part entries are in units of Ms*V (exchange: in units of Ms*V as well, see k_energy).
__global__ void k_energy_finish(const double* __restrict__ part, int nb, double MsV, double lam, double area, int N,
                                double E_ref, double* __restrict__ J, double* __restrict__ en,
                                double* __restrict__ coef_out) {
    __shared__ double red[5][256];
    double s[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        for (int q = 0; q < 5; ++q) s[q] += part[5 * b + q];
    for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ex = red[0][0] * MsV, d = red[1][0] * MsV, z = red[2][0] * MsV, an = red[3][0] * MsV;
        const double mean = red[4][0] / N;
        if (en) {
            en[0] = ex;
            en[1] = d;
            en[2] = z;
            en[3] = an;
            en[4] = ex + d + z + an;
        }
        if (J) *J = (ex + d) / E_ref + lam * (mean - area) * (mean - area);
        *coef_out = 2.0 * lam * (mean - area) / N;
    }
}

__global__ void k_add_coef(double* __restrict__ g, const double* __restrict__ coef, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] += *coef;
}

__global__ void k_port_finish(const double* __restrict__ part, int nb, double inv1, double inv2, double invW,
                              double* __restrict__ J) {
    __shared__ double red[2][256];
    double s1 = 0.0, s2 = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        s1 += part[2 * b];
        s2 += part[2 * b + 1];
    }
    red[0][threadIdx.x] = s1;
    red[1][threadIdx.x] = s2;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *J = invW * (red[0][0] * inv1 - red[1][0] * inv2);
}

template <typename T>
__global__ void k_adj_init(const KParams<T> p, const T* __restrict__ dJdm, const T* __restrict__ mN,
                           const uint8_t* __restrict__ port1, const uint8_t* __restrict__ port2, T src1, T src2,
                           T* __restrict__ lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const int N = p.N;
    V3<T> l = dJdm ? ld3(dJdm, N, i) : v3<T>(0, 0, 0);
    if (port1) {
        const T src = (port1[i] ? src1 : (T)0) - (port2[i] ? src2 : (T)0);
        l.y = l.y + src * mN[N + i];
    }
    st3(lam, N, i, l);
}

template <typename T>
__global__ void k_psi_grad_out(int n, const double* __restrict__ gacc, const double* __restrict__ expl,
                               double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = gacc[i] + (expl ? expl[i] : 0.0);
}

__global__ void k_zero_f64(double* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_stage_fwd(const KParams<T>& p, const StageFwdArgs<T>& a, const cplx<T>* twx, const LocalLaunch& L,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_stage_fwd<T>, dim3(L.blocks), dim3(L.threads), L.lds, s, p, a, twx);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_stage_bwd(const KParams<T>& p, const StageBwdArgs<T>& a, const cplx<T>* twx, const LocalLaunch& L,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_stage_bwd<T>, dim3(L.blocks), dim3(L.threads), L.lds, s, p, a, twx);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_col_conv(const KParams<T>& p, cplx<T>* S, const T* nhat, const cplx<T>* twy, const cplx<T>* twz,
                           const ColLaunch& L, hipStream_t s) {
    if (p.nz == 1)
        hipLaunchKernelGGL((k_col_conv<T, 1>), dim3(L.blocks), dim3(L.threads), L.lds, s, p, S, nhat, twy, twz, L.tk);
    else if (p.nz == 2)
        hipLaunchKernelGGL((k_col_conv<T, 2>), dim3(L.blocks), dim3(L.threads), L.lds, s, p, S, nhat, twy, twz, L.tk);
    else if (p.nz <= 4)
        hipLaunchKernelGGL((k_col_conv<T, 4>), dim3(L.blocks), dim3(L.threads), L.lds, s, p, S, nhat, twy, twz, L.tk);
    else
        hipLaunchKernelGGL((k_col_conv<T, 8>), dim3(L.blocks), dim3(L.threads), L.lds, s, p, S, nhat, twy, twz, L.tk);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_levelset(const KParams<T>& p, const T* phi, const T* psi_fixed, const uint8_t* design, double a,
                           int extrude, T* psi_out, hipStream_t s) {
    hipLaunchKernelGGL(k_levelset<T>, dim3((p.N + 255) / 256), dim3(256), 0, s, p, phi, psi_fixed, design, (T)a,
                       extrude, psi_out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_levelset_vjp(const KParams<T>& p, const T* phi, const double* g, const uint8_t* design, double a,
                               int extrude, double* out, hipStream_t s) {
    const int M = extrude ? p.nx * p.ny : p.N;
    hipLaunchKernelGGL(k_levelset_vjp<T>, dim3((M + 255) / 256), dim3(256), 0, s, p, phi, g, design, a, extrude, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_energy(const KParams<T>& p, double t, const T* psi, const T* m, const cplx<T>* S, const cplx<T>* twx,
                         const uint8_t* antenna, double scale, T* dJdm, double* dJdpsi, double* part,
                         const LocalLaunch& L, hipStream_t s) {
    hipLaunchKernelGGL(k_energy<T>, dim3(L.blocks), dim3(L.threads), L.lds, s, p, t, psi, m, S, twx, antenna,
                       scale, dJdm, dJdpsi, part);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_port_finish(const double* part, int nblocks, double inv1, double inv2, double invW, double* J,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_port_finish, dim3(1), dim3(256), 0, s, part, nblocks, inv1, inv2, invW, J);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_init(const KParams<T>& p, const T* dJdm_T, const T* mN, const uint8_t* port1,
                           const uint8_t* port2, T src1, T src2, T* lam, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_init<T>, dim3((p.N + 255) / 256), dim3(256), 0, s, p, dJdm_T, mN, port1, port2, src1,
                       src2, lam);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_psi_grad_out(const KParams<T>& p, const double* gacc, const double* expl, double* out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_psi_grad_out<T>, dim3((p.N + 255) / 256), dim3(256), 0, s, p.N, gacc, expl, out);
    return hipGetLastError();
}
hipError_t launch_zero_f64(double* ptr, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ptr, n);
    return hipGetLastError();
}

// energy finish needs Ms*V and the objective constants; declared here for the runtime
hipError_t launch_energy_finish_raw(const double* part, int nb, double MsV, double lam, double area, int N,
                                    double E_ref, double* J, double* en, double* coef, double* dJdpsi,
                                    hipStream_t s) {
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(256), 0, s, part, nb, MsV, lam, area, N, E_ref, J, en, coef);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dJdpsi) {
        hipLaunchKernelGGL(k_add_coef, dim3((N + 255) / 256), dim3(256), 0, s, dJdpsi, coef, N);
        e = hipGetLastError();
    }
    return e;
}

hipError_t set_lds_limits(int bytes) {
    hipError_t e = hipSuccess;
#define LLG_ATTR(K) \
    if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void*>(K), hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    LLG_ATTR(k_stage_fwd<float>) LLG_ATTR(k_stage_fwd<double>)
    LLG_ATTR(k_stage_bwd<float>) LLG_ATTR(k_stage_bwd<double>)
    LLG_ATTR((k_col_conv<float, 1>)) LLG_ATTR((k_col_conv<float, 2>)) LLG_ATTR((k_col_conv<float, 4>))
    LLG_ATTR((k_col_conv<float, 8>)) LLG_ATTR((k_col_conv<double, 1>)) LLG_ATTR((k_col_conv<double, 2>))
    LLG_ATTR((k_col_conv<double, 4>)) LLG_ATTR((k_col_conv<double, 8>))
    LLG_ATTR(k_energy<float>) LLG_ATTR(k_energy<double>)
#undef LLG_ATTR
    return e;
}

#define LLG_INST(T)                                                                                                   \
    template hipError_t launch_stage_fwd<T>(const KParams<T>&, const StageFwdArgs<T>&, const cplx<T>*,                \
                                            const LocalLaunch&, hipStream_t);                                         \
    template hipError_t launch_stage_bwd<T>(const KParams<T>&, const StageBwdArgs<T>&, const cplx<T>*,                \
                                            const LocalLaunch&, hipStream_t);                                         \
    template hipError_t launch_col_conv<T>(const KParams<T>&, cplx<T>*, const T*, const cplx<T>*, const cplx<T>*,     \
                                           const ColLaunch&, hipStream_t);                                            \
    template hipError_t launch_levelset<T>(const KParams<T>&, const T*, const T*, const uint8_t*, double, int, T*,    \
                                           hipStream_t);                                                              \
    template hipError_t launch_levelset_vjp<T>(const KParams<T>&, const T*, const double*, const uint8_t*, double,    \
                                               int, double*, hipStream_t);                                            \
    template hipError_t launch_energy<T>(const KParams<T>&, double, const T*, const T*, const cplx<T>*,               \
                                         const cplx<T>*, const uint8_t*, double, T*, double*, double*,                \
                                         const LocalLaunch&, hipStream_t);                                            \
    template hipError_t launch_port_finish<T>(const double*, int, double, double, double, double*, hipStream_t);      \
    template hipError_t launch_adj_init<T>(const KParams<T>&, const T*, const T*, const uint8_t*, const uint8_t*, T,   \
                                           T, T*, hipStream_t);                                                       \
    template hipError_t launch_psi_grad_out<T>(const KParams<T>&, const double*, const double*, double*, hipStream_t);

LLG_INST(float)
LLG_INST(double)

}  // namespace llg
