// Device kernels of the level-set LLG forward / adjoint path (gfx950).
//
// Data layout (all in HBM, component-major SoA, x fastest):
//   vector fields  v[c*N + (iz*ny + iy)*nx + ix]
//   x-spectrum     S[((c*ktiles + t)*nrows + row)*TW + o], row = iz*ny + iy, bin kx = t*TW + o in [0, Px/2]
//   tensor spectrum nhat[(t*NR + (comp*Kz2 + kz)*Ky2 + ky)*TW + o]  (real), NR = ncomp*Kz2*Ky2
//   (TW = 128-byte tile of complex bins: 16 in float, 8 in double)
//
// Demag field B_d = -mu0 Ms N * (psi m) is a linear convolution computed with
// zero padding: a real-to-complex FFT along x of each grid row (fused into the
// local kernel that produced the row), one column kernel that transforms along
// y (and z), multiplies by the tensor spectrum and transforms back, and the
// inverse x FFT fused into the next local kernel.  Three real rows are packed
// into complex signals (x,y components of one row; z components of two rows),
// so every row FFT is a complex FFT of length Px.  All FFTs are radix-4/2
// Stockham passes in LDS with precomputed float64-accurate twiddles.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

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
// LDS arrays of complex values are padded by one element per 2^kLdsPadShift
// (lp maps the logical index to the stored one).  The passes write with
// strides of R or R*Ns elements; without the pad those land in one bank group,
// with it the lanes of a wave spread over the banks.
__device__ __forceinline__ int lp(int a) { return a + (a >> kLdsPadShift); }
// For a and b with no common set bit, lp(a + b) = lp(a) + lp(b) (the shift of
// a bitwise union is the union of the shifts): with a row (column) length P a
// power of two and x < P, lp(s P + x) = lp(x) + lp(s P), a lane index plus a
// uniform offset.

// Byte offsets lp(r 2^k) * SZ of the points of a butterfly (r < 16, k < 16),
// one row per k: a pass reads its R offsets with one uniform (scalar) load
// instead of computing them.
template <int SZ> struct alignas(64) LpOffsets {
    int v[16][16];
    constexpr LpOffsets() : v() {
        for (int k = 0; k < 16; ++k)
            for (int r = 0; r < 16; ++r) v[k][r] = ((r << k) + ((r << k) >> kLdsPadShift)) * SZ;
    }
};
__device__ constexpr LpOffsets<8> kLpOff8{};
__device__ constexpr LpOffsets<16> kLpOff16{};
template <int N> struct OffRow {
    int o[N];
};
// the first N offsets of row k, read in 16-byte pieces
template <typename C, int N> __device__ __forceinline__ OffRow<N> lp_offsets(int k) {
    const int* row;
    if constexpr (sizeof(C) == 8) row = kLpOff8.v[k];
    else row = kLpOff16.v[k];
    OffRow<N> r;
    if constexpr (N >= 4) {
#pragma unroll
        for (int i = 0; i < N / 4; ++i) {
            const int4 t = reinterpret_cast<const int4*>(row)[i];
            r.o[4 * i] = t.x, r.o[4 * i + 1] = t.y, r.o[4 * i + 2] = t.z, r.o[4 * i + 3] = t.w;
        }
    } else {
        const int2 t = *reinterpret_cast<const int2*>(row);
        r.o[0] = t.x, r.o[1] = t.y;
    }
    return r;
}

// Signal b occupies logical positions ((b >> l0) << ls1) + (b & (2^l0 - 1)) + (e << l0),
// e in [0, L): contiguous signals 2^ls1 apart (l0 = 0, the rows), or 2^l0
// signals interleaved element by element (the TK bins of a column tile).  Work
// items are ordered with the low l0 bits of the signal index fastest, then the
// butterfly index, so adjacent lanes touch adjacent elements.  Every stride is
// a power of two, so the indices take shifts and masks, no multiplies.
struct SigMap {
    int l0, ls1;
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

// R-point DFT of v whose upper half v[R/2 .. R-1] is zero (decimation in
// frequency, first stage without its additions): X[2k] = DFT_{R/2}(v)[k],
// X[2k+1] = DFT_{R/2}(v[r] w^r)[k], w = exp(-+2 pi i / R).
template <typename C, bool INV, int R>
__device__ __forceinline__ void dft_half_in(C* v) {
    using T = decltype(C().x);
    constexpr int H = R / 2;
    C a[H], b[H];
#pragma unroll
    for (int r = 0; r < H; ++r) {
        a[r] = v[r];
        const int m = r * (16 / R);
        if (m == 0) {
            b[r] = v[r];
        } else if (m == 4) {
            b[r] = INV ? cmul_i(v[r]) : cmul_mi(v[r]);
        } else {
            b[r] = cmul(v[r], cmk<C>((T)kC16[m], INV ? (T)kS16[m] : -(T)kS16[m]));
        }
    }
    dft_small<C, INV, H>(a);
    dft_small<C, INV, H>(b);
#pragma unroll
    for (int k = 0; k < H; ++k) {
        v[2 * k] = a[k];
        v[2 * k + 1] = b[k];
    }
}

// The lower half X[0 .. R/2-1] of the R-point DFT of v (decimation in time,
// last stage without its subtractions): X[k] = E[k] + w^k O[k] with E, O the
// DFTs of the even and odd samples.  X[R/2 ..] is left unset.
template <typename C, bool INV, int R>
__device__ __forceinline__ void dft_half_out(C* v) {
    using T = decltype(C().x);
    constexpr int H = R / 2;
    C e[H], o[H];
#pragma unroll
    for (int r = 0; r < H; ++r) {
        e[r] = v[2 * r];
        o[r] = v[2 * r + 1];
    }
    dft_small<C, INV, H>(e);
    dft_small<C, INV, H>(o);
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const int m = k * (16 / R);
        C t;
        if (m == 0) {
            t = o[k];
        } else if (m == 4) {
            t = INV ? cmul_i(o[k]) : cmul_mi(o[k]);
        } else {
            t = cmul(o[k], cmk<C>((T)kC16[m], INV ? (T)kS16[m] : -(T)kS16[m]));
        }
        v[k] = cadd(e[k], t);
    }
}

// One Stockham pass of radix R over nsig signals of length L = 2^lL (in place
// via registers).  Requires nsig * L <= MAXREG * blockDim.x.
// A butterfly reads its R points at a0 + r 2^k and writes them at b0 + r 2^ko,
// where a0 has no bit set in [k, k + log2 R) and b0 none in [ko, ko + log2 R).
// For disjoint bit sets (A + X) >> s = (A >> s) + (X >> s), so the pad splits
// exactly: lp(A + X) = lp(A) + lp(X), one lane address plus a
// block-uniform offset per point.
template <typename C, bool INV, int R, int MAXREG, bool OPQ = true>
__device__ __forceinline__ void fft_pass(C* buf, const SigMap sm, int lL, int lNs, int nsig, const C* __restrict__ tw) {
    constexpr int IPT = MAXREG / R;
    constexpr int LR = ilog2(R);
    const int lnbf = lL - LR;
    const int total = nsig << lnbf;
    // work item it: signal / butterfly bits below k = l0 + lnbf, the rest the
    // signal group; its R inputs lie 2^k apart
    const int k = sm.l0 + lnbf;
    const int mk = (1 << k) - 1, m0 = (1 << sm.l0) - 1;
    const OffRow<R> ol = lp_offsets<C, R>(k);
    // OPQ: the thread index, opaque to the compiler.  Without it the compiler
    // hoists every radix variant's lane addresses out of the caller's pass loop,
    // computing (and holding registers for) those of radices that never run; a
    // caller whose registers sit just below an occupancy step keeps the hoisting
    int tid = (int)threadIdx.x;
    if constexpr (OPQ) asm volatile("" : "+v"(tid));
    C v[IPT][R];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int it = tid + q * blockDim.x;
        if (it < total) {
            const char* pb = reinterpret_cast<const char*>(buf + lp(((it >> k) << sm.ls1) + (it & mk)));
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = *reinterpret_cast<const C*>(pb + ol.o[r]);
        }
    }
    __syncthreads();
    const int lstride = lL - lNs - LR;  // twiddle index step L / (Ns R)
    const int ko = lNs + sm.l0;         // outputs lie 2^ko apart
    const OffRow<R> os = lp_offsets<C, R>(ko);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int it = tid + q * blockDim.x;
        if (it < total) {
            const int j = (it >> sm.l0) & ((1 << lnbf) - 1);
            const int jm = j & ((1 << lNs) - 1);
            // the first pass (Ns = 1) has every twiddle equal to 1: skipped (a product with exactly 1 is exact)
            if (lNs > 0) {
                // twiddle r sits r u bytes into the table, u = (jm << lstride) sizeof(C) < 2^24
                const unsigned u = (unsigned)(jm << lstride) * (unsigned)sizeof(C);
                const char* tb = reinterpret_cast<const char*>(tw);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = *reinterpret_cast<const C*>(tb + __umul24((unsigned)r, u));
                    if (INV) w = cconj(w);
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            dft_small<C, INV, R>(v[q]);
            const int b0 = ((it >> k) << sm.ls1) + (it & m0) + ((((j - jm) << LR) + jm) << sm.l0);
            char* pb = reinterpret_cast<char*>(buf + lp(b0));
#pragma unroll
            for (int r = 0; r < R; ++r) *reinterpret_cast<C*>(pb + os.o[r]) = v[q][r];
        }
    }
    __syncthreads();
}

// Full FFT of length L (power of two) of nsig signals; tw = exp(-2 pi i k / L).
// Passes of the largest radix the register budget allows (16 in float, 8 in
// double) while enough points remain, then one pass of the remaining radix.
template <typename C, bool INV, int MAXREG, bool OPQ = true>
__device__ __forceinline__ void fft_lds(C* buf, const SigMap sm, int L, int nsig, const C* __restrict__ tw) {
    int lL = 0;
    while ((1 << lL) < L) ++lL;
    int lNs = 0;
    while (lNs < lL) {
        const int rem = lL - lNs;
        if constexpr (MAXREG >= 16) {
            if (rem >= 4) {
                fft_pass<C, INV, 16, MAXREG, OPQ>(buf, sm, lL, lNs, nsig, tw);
                lNs += 4;
                continue;
            }
        }
        if constexpr (MAXREG >= 8) {
            if (rem >= 3) {
                fft_pass<C, INV, 8, MAXREG, OPQ>(buf, sm, lL, lNs, nsig, tw);
                lNs += 3;
                continue;
            }
        }
        if (rem >= 2) {
            fft_pass<C, INV, 4, MAXREG, OPQ>(buf, sm, lL, lNs, nsig, tw);
            lNs += 2;
        } else {
            fft_pass<C, INV, 2, MAXREG, OPQ>(buf, sm, lL, lNs, nsig, tw);
            lNs += 1;
        }
    }
}

template <typename T> struct MaxReg;
template <> struct MaxReg<float> { static constexpr int v = 16; };
template <> struct MaxReg<double> { static constexpr int v = 8; };

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
// 1/s: the hardware reciprocal in float (1 ulp), a correctly rounded division in double
template <typename T> __device__ __forceinline__ T recip(T s) {
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(s);
    else return (T)1 / s;
}
// Knuth's error-free two-sum: s = fl(x + y) and x + y = s + e exactly
template <typename T> __device__ __forceinline__ T two_sum(T x, T y, T& e) {
    const T s = x + y;
    const T bp = s - x;
    const T ap = s - bp;
    e = (x - ap) + (y - bp);
    return s;
}

// The buffers behind the tables and launch descriptors are device global
// memory.  Accessing them through global-space pointers gives global rather
// than flat memory instructions: a scalar base with a 32-bit offset, and loads
// whose completion the LDS waits do not have to drain.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* glb(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
// complex values and 16-byte units move as plain vectors (the HIP vector
// classes do not bind to global-space references)
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
using vec4 = T __attribute__((ext_vector_type(4)));
// a load at an unsigned 32-bit byte offset from a block-uniform base (the
// scalar-base addressing form: no 64-bit address arithmetic per lane)
template <typename T>
__device__ __forceinline__ T gld_at(const T* base, unsigned byte_off) {
    return *(const __attribute__((address_space(1))) T*)((const __attribute__((address_space(1))) char*)base + byte_off);
}
template <typename T>
__device__ __forceinline__ void gst_at(T* base, unsigned byte_off, T v) {
    *(__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)base + byte_off) = v;
}
// element i (0 <= i < 2^28) of a per-instance node array: a lane byte offset from
// the block-uniform base
template <typename T>
__device__ __forceinline__ T gat(const T* base, int i) {
    return gld_at(base, (unsigned)i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void gput(T* base, int i, T v) {
    gst_at(base, (unsigned)i * (unsigned)sizeof(T), v);
}
template <typename C>
__device__ __forceinline__ C gldc_at(const C* base, unsigned byte_off) {
    using T = decltype(C().x);
    const vec2<T> v = *(const __attribute__((address_space(1))) vec2<T>*)((const __attribute__((address_space(1))) char*)base + byte_off);
    return cmk<C>(v.x, v.y);
}
template <typename C>
__device__ __forceinline__ void gstc_at(C* base, unsigned byte_off, C c) {
    using T = decltype(C().x);
    vec2<T> v;
    v.x = c.x;
    v.y = c.y;
    *(__attribute__((address_space(1))) vec2<T>*)((__attribute__((address_space(1))) char*)base + byte_off) = v;
}
template <typename C>
__device__ __forceinline__ C gld(const C* p) {
    using T = decltype(C().x);
    const vec2<T> v = *(const __attribute__((address_space(1))) vec2<T>*)p;
    return cmk<C>(v.x, v.y);
}
template <typename C>
__device__ __forceinline__ void gst(C* p, C c) {
    using T = decltype(C().x);
    vec2<T> v;
    v.x = c.x;
    v.y = c.y;
    *(__attribute__((address_space(1))) vec2<T>*)p = v;
}

template <typename T> __device__ __forceinline__ V3<T> ld3(const T* __restrict__ v, int N, int i) {
    const auto g = glb(v);
    return v3(g[i], g[N + i], g[2 * N + i]);
}
template <typename T> __device__ __forceinline__ void st3(T* __restrict__ v, int N, int i, V3<T> a) {
    const auto g = glb(v);
    g[i] = a.x;
    g[N + i] = a.y;
    g[2 * N + i] = a.z;
}
// The same with one lane byte offset (i < N <= 2^28, so i sizeof(T) < 2^32) from
// three block-uniform component bases: fewer registers where many node vectors
// are held at once (the backward stage's inputs), but a neighbour's +-1 cannot
// fold into the instruction's offset, so stencil reads keep the indexed form.
template <typename T> __device__ __forceinline__ V3<T> ld3u(const T* __restrict__ v, int N, int i) {
    const unsigned o = (unsigned)i * (unsigned)sizeof(T);
    return v3(gld_at(v, o), gld_at(v + N, o), gld_at(v + 2 * (size_t)N, o));
}
template <typename T> __device__ __forceinline__ void st3u(T* __restrict__ v, int N, int i, V3<T> a) {
    const unsigned o = (unsigned)i * (unsigned)sizeof(T);
    gst_at(v, o, a.x);
    gst_at(v + N, o, a.y);
    gst_at(v + 2 * (size_t)N, o, a.z);
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

// Drive waveform: sin(2 pi f1 t), switching to f2 at t_switch > 0 with a
// continuous phase; without a switch and with f2 > 0 the two-tone excitation
// sin(2 pi f1 t) + sin(2 pi f2 t); kind 1: the linear ramp t / t_ramp.
__device__ __forceinline__ double drive_value(double f1, double f2, double tsw, int kind, double t_ramp, double t) {
    const double twopi = 6.283185307179586476925286766559;
    if (kind == 1) return t / t_ramp;
    if (tsw <= 0.0 && f2 > 0.0) return sin(twopi * f1 * t) + sin(twopi * f2 * t);
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
    constexpr int TW = spec_tile<T>();
    const int Px = p.Px;
    const unsigned cb = (unsigned)((size_t)p.ktiles * p.nrows * TW * sizeof(C));  // component stride in bytes
    for (int k = threadIdx.x; k < Px; k += blockDim.x) {
        const bool cj = k > Px / 2;
        const int kk = cj ? Px - k : k;
        const unsigned o = ((unsigned)(kk / TW) * (unsigned)p.nrows + (unsigned)r0) * 128u + (unsigned)(kk % TW) * (unsigned)sizeof(C);
        C ax = gldc_at(S, o), ay = gldc_at(S, o + cb), az = gldc_at(S, o + 2 * cb);
        C bx = cmk<C>(0, 0), by = bx, bz = bx;
        if (v1) {
            bx = gldc_at(S, o + 128u);
            by = gldc_at(S, o + 128u + cb);
            bz = gldc_at(S, o + 128u + 2 * cb);
        }
        if (cj) {
            ax = cconj(ax); ay = cconj(ay); az = cconj(az);
            bx = cconj(bx); by = cconj(by); bz = cconj(bz);
        }
        Z[lp(k)] = cadd(ax, cmul_i(ay));
        Z[lp(k) + lp(Px)] = cadd(bx, cmul_i(by));
        Z[lp(k) + lp(2 * Px)] = cadd(az, cmul_i(bz));
    }
}

template <typename T>
__device__ __forceinline__ void pack_lds_to_rows(const KParams<T>& p, cplx<T>* __restrict__ S, int r0, bool v1,
                                                 const cplx<T>* Z) {
    using C = cplx<T>;
    constexpr int TW = spec_tile<T>();
    const int Px = p.Px, Kx = p.Kx;
    const unsigned cb = (unsigned)((size_t)p.ktiles * p.nrows * TW * sizeof(C));  // component stride in bytes
    const T h = (T)0.5;
    for (int k = threadIdx.x; k < Kx; k += blockDim.x) {
        const int kn = (Px - k) & (Px - 1);
        C out[6];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const C a = Z[lp(k) + lp(s * Px)];
            const C b = cconj(Z[lp(kn) + lp(s * Px)]);
            const C sum = cadd(a, b), dif = csub(a, b);
            out[2 * s] = cmk<C>(h * sum.x, h * sum.y);       // spectrum of the real part
            out[2 * s + 1] = cmk<C>(h * dif.y, -h * dif.x);  // spectrum of the imaginary part
        }
        const unsigned o = ((unsigned)(k / TW) * (unsigned)p.nrows + (unsigned)r0) * 128u + (unsigned)(k % TW) * (unsigned)sizeof(C);
        gstc_at(S, o, out[0]);
        gstc_at(S, o + cb, out[1]);
        gstc_at(S, o + 2 * cb, out[4]);
        if (v1) {
            gstc_at(S, o + 128u, out[2]);
            gstc_at(S, o + 128u + cb, out[3]);
            gstc_at(S, o + 128u + 2 * cb, out[5]);
        }
    }
}

// ---------------------------------------------------------------------------
// shared-memory layout of the local (row-pair) kernels
//   Z  [3 * Px] complex  three packed row signals (demag only; padded, see lp)
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
    L.Tw = L.Z + (demag ? lds_pad(3 * Px) : 0);
    L.R = reinterpret_cast<T*>(L.Tw + (demag ? Px : 0));
    return L;
}

// ---------------------------------------------------------------------------
// batched staging of global data into LDS
// ---------------------------------------------------------------------------
// Up to three independent copy streams (element e of stream k: value ldk(e),
// stored by stk(e, value)) advance in chunks of U_k elements per thread; all
// loads of a chunk, across the streams, are issued before the first of them
// is waited on, so a block pays about one memory latency per chunk instead
// of one per loop iteration.
template <typename V, int U>
struct Regs {
    V v[U];
};

template <int UA, int UB, int UC, typename VA, typename VB, typename VC, class LA, class SA, class LB, class SB, class LC,
          class SC>
__device__ __forceinline__ void gather3(int na, LA&& la, SA&& sa, int nb, LB&& lb, SB&& sb, int nc, LC&& lc, SC&& sc) {
    const int bd = blockDim.x;
    int ea = threadIdx.x, eb = threadIdx.x, ec = threadIdx.x;
    while (ea < na || eb < nb || ec < nc) {
        Regs<VA, UA> ra;
        Regs<VB, UB> rb;
        Regs<VC, UC> rc;
#pragma unroll
        for (int u = 0; u < UA; ++u)
            if (ea + u * bd < na) ra.v[u] = la(ea + u * bd);
#pragma unroll
        for (int u = 0; u < UB; ++u)
            if (eb + u * bd < nb) rb.v[u] = lb(eb + u * bd);
#pragma unroll
        for (int u = 0; u < UC; ++u)
            if (ec + u * bd < nc) rc.v[u] = lc(ec + u * bd);
#pragma unroll
        for (int u = 0; u < UA; ++u)
            if (ea + u * bd < na) sa(ea + u * bd, ra.v[u]);
#pragma unroll
        for (int u = 0; u < UB; ++u)
            if (eb + u * bd < nb) sb(eb + u * bd, rb.v[u]);
#pragma unroll
        for (int u = 0; u < UC; ++u)
            if (ec + u * bd < nc) sc(ec + u * bd, rc.v[u]);
        ea += UA * bd;
        eb += UB * bd;
        ec += UC * bd;
    }
}

// Inputs of a row-pair block, staged together:
//   rows  r0-1 .. r0+2 of NV node arrays src[v] (component comp[v]) into R,
//         rows outside the grid left unset (never read);
//   the packed spectrum of rows r0, r0+1 (inverse-FFT input) into Z;
//   the x twiddles into Tw.
// SB: the staged rows are read at lane byte offsets from block-uniform bases
// (fewer registers for the loads in flight; the backward kernel holds 28 of them)
template <typename T, int NV, bool SB = false>
__device__ __forceinline__ void stage_inputs(const KParams<T>& p, int r0, bool v1, bool rows, int nvu,
                                             const T* const (&src)[NV], const int (&comp)[NV], T* R,
                                             const cplx<T>* __restrict__ S, cplx<T>* Z,
                                             const cplx<T>* __restrict__ tw, cplx<T>* Tw) {
    using C = cplx<T>;
    struct Node {
        T v[4][NV];  // rows r0-1 .. r0+2 at one x
    };
    struct Bin {
        C a[3], b[3];
    };
    constexpr int TW = spec_tile<T>();
    const int nx = p.nx, Px = p.Px, N = p.N, nrows = p.nrows;
    const size_t cs = (size_t)p.ktiles * nrows * TW;
    const int nrow_el = rows ? nx : 0;
    const int nspec = S ? Px : 0;
    const int ntw = tw ? Px : 0;
    auto lrow = [&](int x) {
        Node n;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 - 1 + q;
            if (r >= 0 && r < nrows) {
                const int i = r * nx + x;
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v < nvu) {
                        if constexpr (SB) n.v[q][v] = gat(src[v] + (size_t)comp[v] * N, i);
                        else n.v[q][v] = glb(src[v])[comp[v] * N + i];
                    }
            }
        }
        return n;
    };
    auto srow = [&](int x, const Node& n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 - 1 + q;
            if (r >= 0 && r < nrows) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v < nvu) R[(q * nvu + v) * nx + x] = n.v[q][v];
            }
        }
    };
    const unsigned cb = (unsigned)(cs * sizeof(C));  // component stride in bytes (a spectrum is below 2^32 bytes)
    auto lspec = [&](int k) {
        Bin b;
        const int kk = k > Px / 2 ? Px - k : k;
        const unsigned o = ((unsigned)(kk / TW) * (unsigned)nrows + (unsigned)r0) * 128u + (unsigned)(kk % TW) * (unsigned)sizeof(C);
        b.a[0] = gldc_at(S, o);
        b.a[1] = gldc_at(S, o + cb);
        b.a[2] = gldc_at(S, o + 2 * cb);
        if (v1) {
            b.b[0] = gldc_at(S, o + 128u);
            b.b[1] = gldc_at(S, o + 128u + cb);
            b.b[2] = gldc_at(S, o + 128u + 2 * cb);
        } else {
            b.b[0] = b.b[1] = b.b[2] = cmk<C>(0, 0);
        }
        return b;
    };
    auto sspec = [&](int k, Bin b) {
        if (k > Px / 2) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                b.a[c] = cconj(b.a[c]);
                b.b[c] = cconj(b.b[c]);
            }
        }
        Z[lp(k)] = cadd(b.a[0], cmul_i(b.a[1]));
        Z[lp(k) + lp(Px)] = cadd(b.b[0], cmul_i(b.b[1]));
        Z[lp(k) + lp(2 * Px)] = cadd(b.a[2], cmul_i(b.b[2]));
    };
    auto ltw = [&](int k) { return gld(tw + k); };
    auto stw = [&](int k, C w) { Tw[k] = w; };
    gather3<1, 1, 1, Node, Bin, C>(nrow_el, lrow, srow, nspec, lspec, sspec, ntw, ltw, stw);
}

// ---------------------------------------------------------------------------
// batch addressing: thread block -> (instance, unit), role -> buffer
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T* role(const InstTab& tb, int id) {
    return id < 0 ? nullptr : static_cast<T*>(tb.b[id]);
}

template <typename T>
__device__ __forceinline__ StageFwdArgs<T> resolve_fwd(const KParams<T>& p, const InstTab& tb, const FwdL& L) {
    StageFwdArgs<T> a;
    const size_t n3 = (size_t)3 * p.N;
    a.stage = L.stage;
    a.t = L.t;
    a.psi = role<T>(tb, B_PSI);
    a.ys = L.ext_ys ? static_cast<const T*>(L.ext_ys) : role<T>(tb, L.ys);
    a.mn = role<T>(tb, L.mn);
    a.acc = role<T>(tb, L.acc);
    a.ynext = L.ext_ynext ? static_cast<T*>(L.ext_ynext) : role<T>(tb, L.ynext);
    a.S = role<cplx<T>>(tb, L.spec);
    a.antenna = p.has_ant ? role<uint8_t>(tb, B_ANT) : nullptr;
    a.ys_store = L.store_j >= 0 ? role<T>(tb, B_YS) + ((size_t)L.store_j * 4 + L.stage) * n3 : nullptr;
    a.Bs_store = L.ext_B ? static_cast<T*>(L.ext_B)
                         : (L.store_j >= 0 ? role<T>(tb, B_BS) + ((size_t)L.store_j * 4 + L.stage) * n3 : nullptr);
    const bool port = L.port && (L.port == 3 || (p.n_p1 + p.n_p2) > 0);
    a.port1 = port ? role<uint8_t>(tb, B_P1) : nullptr;
    a.port2 = port ? role<uint8_t>(tb, B_P2) : nullptr;
    a.port_lin = L.port >= 2 ? L.port - 1 : 0;
    a.port_part = !port ? nullptr
                        : (a.port_lin ? role<double>(tb, B_PSER) + (size_t)L.pstep * 2 * p.nloc
                                      : role<double>(tb, B_PPART));
    a.do_inv = L.do_inv;
    a.do_fwd = L.do_fwd;
    return a;
}

template <typename T>
__device__ __forceinline__ StageBwdArgs<T> resolve_bwd(const KParams<T>& p, const InstTab& tb, const BwdL& L) {
    StageBwdArgs<T> a;
    const size_t n3 = (size_t)3 * p.N;
    const int st = L.stage < 0 ? 0 : L.stage;
    a.stage = L.stage;
    a.psi = role<T>(tb, B_PSI);
    a.ys = L.ext_ys ? static_cast<const T*>(L.ext_ys) : role<T>(tb, B_YS) + ((size_t)L.j * 4 + st) * n3;
    a.Bs = L.ext_B ? static_cast<const T*>(L.ext_B) : role<T>(tb, B_BS) + ((size_t)L.j * 4 + st) * n3;
    a.u_cur = role<T>(tb, L.ucur);
    a.ell = role<T>(tb, B_ELL);
    a.lamp = role<T>(tb, L.lamp);
    a.lacc_in = L.ext_lacc ? nullptr : role<T>(tb, L.lacc);
    a.lacc_out = L.ext_lacc ? static_cast<T*>(L.ext_lacc) : role<T>(tb, L.lacc);
    a.gpsi = role<double>(tb, B_GPSI);
    a.y_prev = L.prev_j < 0 ? nullptr
               : L.ext_ys ? static_cast<const T*>(L.ext_ys)
                          : role<T>(tb, B_YS) + ((size_t)L.prev_j * 4 + L.prev_st) * n3;
    a.u_next = role<T>(tb, L.unext);
    a.S = role<cplx<T>>(tb, B_S);
    const bool port = L.port_src && L.W > 0 && (L.port_lin == 2 || (p.n_p1 + p.n_p2) > 0);
    a.port1 = port ? role<uint8_t>(tb, B_P1) : nullptr;
    a.port2 = port ? role<uint8_t>(tb, B_P2) : nullptr;
    a.src_lin = L.port_lin;
    a.seed_unit = L.seed_unit;
    if (port && L.port_lin) {
        const double* g = role<double>(tb, B_PSRC) + 2 * (size_t)L.pstep;
        a.src1 = (T)g[0];
        a.src2 = (T)g[1];
    } else {
        a.src1 = port && p.n_p1 > 0 ? (T)(2.0 / ((double)L.W * p.n_p1)) : (T)0;
        a.src2 = port && p.n_p2 > 0 ? -(T)(2.0 / ((double)L.W * p.n_p2)) : (T)0;
    }
    a.do_inv = L.do_inv;
    a.do_fwd = L.do_fwd;
    return a;
}

// ---------------------------------------------------------------------------
// forward local kernel: inverse x-FFT (demag) + local field + LL RHS + RK4
// stage update + forward x-FFT of the next stage's magnetisation
// ---------------------------------------------------------------------------
template <typename T, int MR, bool SR, bool LIN = false>
__global__ void __launch_bounds__(512) k_stage_fwd(const BatchArgs<T> ba, const FwdL L) {
    using C = cplx<T>;
    constexpr int NV = 4;  // m_x, m_y, m_z, psi
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][512 / 64];
    const int2 wk = ba.single ? make_int2(0, (int)blockIdx.x) : ba.work[blockIdx.x];
    const KParams<T> p = ba.ptab[wk.x];
    const InstTab& tb = ba.itab[wk.x];
    const StageFwdArgs<T> a = resolve_fwd<T>(p, tb, L);
    const cplx<T>* __restrict__ twx = role<cplx<T>>(tb, B_TWX);
    const int Px = p.Px, nx = p.nx, N = p.N;
    const bool demag_in = a.do_inv != 0, demag_any = (a.do_inv | a.do_fwd) != 0;
    const LocalSmem<T> LS = local_smem<T>(smem_raw, Px, demag_any);
    C* Z = LS.Z;
    T* R = LS.R;
    const int r0 = 2 * wk.y;
    const bool v1 = r0 + 1 < p.nrows;
    const SigMap sm{0, ilog2_rt(Px)};

    // Work items are (row, x) pairs of the two rows, item = rr * nx + x, so a
    // narrow row pair still spreads over twice as many lanes.  The accumulator
    // and step-start state of this thread's first item are requested first, so
    // their latency overlaps the staging and the inverse FFT.
    const int nitem = v1 ? 2 * nx : nx;
    V3<T> pre_acc = v3<T>(0, 0, 0), pre_mn = v3<T>(0, 0, 0), pre_lo = v3<T>(0, 0, 0);
    uint8_t pre_ant = 0, pre_p1 = 0, pre_p2 = 0;
    const bool need_acc = a.stage >= 1 && a.stage <= 3, need_mn = a.stage >= 1 && a.stage <= 3;
    const bool need_lo = sizeof(T) == 4 && a.stage == 3;  // low part of a float state
    if ((int)threadIdx.x < nitem) {
        const int i = r0 * nx + threadIdx.x;  // rows r0, r0+1 are contiguous
        if (need_acc) pre_acc = ld3(a.acc, N, i);
        if (need_mn) pre_mn = ld3(a.mn, N, i);
        if (need_lo) pre_lo = ld3(a.mn + (size_t)3 * N, N, i);
        if (a.antenna) pre_ant = glb(a.antenna)[i];
        if (a.port_part) {
            pre_p1 = glb(a.port1)[i];
            pre_p2 = glb(a.port2)[i];
        }
    }
    // the neighbour rows r0-1 .. r0+2 of y_s and psi go through LDS (SR), or,
    // where that would cost a resident block per CU, are read from memory in place
    constexpr bool srows = SR;
    {
        const T* const src[NV] = {a.ys, a.ys, a.ys, a.psi};
        const int comp[NV] = {0, 1, 2, 0};
        stage_inputs<T, NV>(p, r0, v1, srows, NV, src, comp, R, demag_in ? a.S : nullptr, Z,
                            demag_any ? twx : nullptr, LS.Tw);
    }
    __syncthreads();
    if (demag_in) fft_lds<C, true, MR>(Z, sm, Px, 3, LS.Tw);

    const T drv = ((p.terms & 4) && a.antenna) ? (T)drive_value(p.f1, p.f2, p.t_switch, p.drive_kind, p.t_ramp, a.t) : (T)0;
    const T dt = p.dt;
    const int iy0 = r0 % p.ny, iz0 = r0 / p.ny;
    double s1 = 0.0, s2 = 0.0;
    for (int it = threadIdx.x; it < nitem; it += blockDim.x) {
        {
            const int rr = it >= nx ? 1 : 0;
            const int x = it - rr * nx;
            const int r = r0 + rr;
            const int q = rr + 1;
            int iy = iy0 + rr, iz = iz0;
            if (iy == p.ny) iy = 0, iz += 1;
            const int i = r * nx + x;
            auto RM = [&](int qq, int xx) {
                if constexpr (!SR) return ld3(a.ys, N, (r0 - 1 + qq) * nx + xx);
                else return v3<T>(R[(qq * NV + 0) * nx + xx], R[(qq * NV + 1) * nx + xx], R[(qq * NV + 2) * nx + xx]);
            };
            auto RP = [&](int qq, int xx) {
                if constexpr (!SR) return glb(a.psi)[(r0 - 1 + qq) * nx + xx];
                else return R[(qq * NV + 3) * nx + xx];
            };
            const V3<T> m = RM(q, x);
            const T pi = RP(q, x);
            V3<T> B = v3<T>(0, 0, 0);
            if (demag_in) {
                const C z01 = Z[lp(x) + lp(rr * Px)];
                const C z2 = Z[lp(x) + lp(2 * Px)];
                B = v3<T>(z01.x, z01.y, rr == 0 ? z2.x : z2.y);
            }
            if (p.terms & 1) {
                // exchange: sum_j exw_d psi_j/(psi_i+psi_j) (m_j - m_i), free ends
                V3<T> Be = v3<T>(0, 0, 0);
                auto add = [&](V3<T> mj, T pj, T w) {
                    const T s = pi + pj;
                    if (s != (T)0) Be = Be + (w * pj * recip(s)) * (mj - m);
                };
                if (x > 0) add(RM(q, x - 1), RP(q, x - 1), p.exw[0]);
                if (x < nx - 1) add(RM(q, x + 1), RP(q, x + 1), p.exw[0]);
                if (iy > 0) add(RM(q - 1, x), RP(q - 1, x), p.exw[1]);
                if (iy < p.ny - 1) add(RM(q + 1, x), RP(q + 1, x), p.exw[1]);
                if (iz > 0) add(ld3(a.ys, N, i - nx * p.ny), glb(a.psi)[i - nx * p.ny], p.exw[2]);
                if (iz < p.nz - 1) add(ld3(a.ys, N, i + nx * p.ny), glb(a.psi)[i + nx * p.ny], p.exw[2]);
                B = B + Be;
            }
            if (p.terms & 4) {
                B = B + v3<T>(p.B0[0], p.B0[1], p.B0[2]);
                const bool ant = a.antenna && (it == (int)threadIdx.x ? pre_ant : glb(a.antenna)[i]);
                if (ant) B = B + drv * v3<T>(p.brf[0], p.brf[1], p.brf[2]);
            }
            if (p.terms & 8) {
                const V3<T> u = v3<T>(p.u[0], p.u[1], p.u[2]);
                B = B + (p.anis * dot(m, u)) * u;
            }
            V3<T> f = v3<T>(0, 0, 0);
            if (pi > p.psi_freeze) {  // psi >= 0: with psi_freeze = 0 every node but psi = 0 moves
                const T al = node_alpha(p, x, iy, iz);
                const T gp = p.gamma / ((T)1 + al * al);
                const V3<T> c = cross(m, B);
                f = (-gp) * (c + al * cross(m, c));
            }
            if (a.ys_store) st3(a.ys_store, N, i, m);
            if (a.Bs_store) st3(a.Bs_store, N, i, B);
            const bool first = it == (int)threadIdx.x;
            const V3<T> accv = need_acc ? (first ? pre_acc : ld3(a.acc, N, i)) : v3<T>(0, 0, 0);
            const V3<T> mnv = need_mn ? (first ? pre_mn : ld3(a.mn, N, i)) : v3<T>(0, 0, 0);
            V3<T> yn;
            if (a.stage == -3) {
                yn = m;  // prologue: spectrum of psi * m only
            } else if (a.stage < 0) {
                yn = f;  // field evaluation: rhs out
            } else if (a.stage == 0) {
                // acc holds the step's increment dt/6 (k1 + 2 k2 + 2 k3), added to m_n once at stage 3:
                // one rounding of the O(1) state per step instead of four
                st3(a.acc, N, i, (dt / (T)6) * f);
                yn = m + (dt / (T)2) * f;
            } else if (a.stage == 1) {
                st3(a.acc, N, i, accv + (dt / (T)3) * f);
                yn = mnv + (dt / (T)2) * f;
            } else if (a.stage == 2) {
                st3(a.acc, N, i, accv + (dt / (T)3) * f);
                yn = mnv + dt * f;
            } else if constexpr (sizeof(T) == 4) {
                // float state kept as hi + lo (lo at offset 3N of the state buffer): m_{n+1} = hi + (lo + increment)
                // by an error-free two-sum, so that rounding to float does not accumulate over the steps
                const V3<T> d = accv + (dt / (T)6) * f;
                const V3<T> lo = first ? pre_lo : ld3(a.mn + (size_t)3 * N, N, i);
                V3<T> e;
                yn = v3<T>(two_sum(mnv.x, d.x + lo.x, e.x), two_sum(mnv.y, d.y + lo.y, e.y),
                           two_sum(mnv.z, d.z + lo.z, e.z));
                st3(a.ynext + (size_t)3 * N, N, i, e);
            } else {
                yn = mnv + (accv + (dt / (T)6) * f);
            }
            if (a.ynext) st3(a.ynext, N, i, yn);
            if constexpr (LIN) {
                // next stage state of an embedded Runge-Kutta step: the same fused multiply-adds, in the same
                // order, as the stage-sum kernel, so that both give the same bits
                const auto g = [&](const void* q) { return ld3(static_cast<const T*>(q), N, i); };
                V3<T> y = g(L.lin_base);
                for (int j = 0; j < L.lin_nt; ++j) {
                    const V3<T> sj = g(L.lin_src[j]);
                    const T c = (T)L.lin_c[j];
                    y = v3<T>(fma(c, sj.x, y.x), fma(c, sj.y, y.y), fma(c, sj.z, y.z));
                }
                const T cf = (T)L.lin_cf;
                y = v3<T>(fma(cf, yn.x, y.x), fma(cf, yn.y, y.y), fma(cf, yn.z, y.z));
                st3(static_cast<T*>(L.lin_out), N, i, y);
                yn = y;  // the transform below takes psi * Y'
            }
            if (a.port_part) {
                if (a.port_lin == 2) {
                    s1 += (double)pi * (double)yn.x;  // curve objective: psi m_x and psi over every node
                    s2 += (double)pi;
                } else {
                    const double v = a.port_lin ? (double)yn.y : (double)yn.y * (double)yn.y;
                    const bool first_it = it == (int)threadIdx.x;
                    if (first_it ? pre_p1 : glb(a.port1)[i]) s1 += v;
                    if (first_it ? pre_p2 : glb(a.port2)[i]) s2 += v;
                }
            }
            if (a.do_fwd) {
                // packed forward-FFT input: (x, y) of each row, z of row 0 + i z of row 1
                T* zr = reinterpret_cast<T*>(Z);
                Z[lp(x) + lp(rr * Px)] = cmk<C>(pi * yn.x, pi * yn.y);
                zr[2 * (lp(x) + lp(2 * Px)) + rr] = pi * yn.z;
                if (!v1) {
                    Z[lp(x) + lp(Px)] = cmk<C>(0, 0);
                    zr[2 * (lp(x) + lp(2 * Px)) + 1] = (T)0;
                }
            }
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
            if (a.port_lin) {
                glb(a.port_part)[2 * wk.y] = t1;
                glb(a.port_part)[2 * wk.y + 1] = t2;
            } else {
                glb(a.port_part)[2 * wk.y] += t1;
                glb(a.port_part)[2 * wk.y + 1] += t2;
            }
        }
    }
    if (a.do_fwd) {
        for (int x = nx + threadIdx.x; x < Px; x += blockDim.x) {
            Z[lp(x)] = cmk<C>(0, 0);
            Z[lp(x) + lp(Px)] = cmk<C>(0, 0);
            Z[lp(x) + lp(2 * Px)] = cmk<C>(0, 0);
        }
        __syncthreads();
        fft_lds<C, false, MR>(Z, sm, Px, 3, LS.Tw);
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
    if (!(psi_i > p.psi_freeze)) return v3<T>(0, 0, 0);  // frozen node: no dynamics to transpose
    const T al = node_alpha(p, ix, iy, iz);
    const T gp = p.gamma / ((T)1 + al * al);
    const V3<T> w = cross(ell, m);
    return (-gp) * (w + al * cross(w, m));
}

// Per-node inputs of a backward stage, loaded together so that one memory
// latency covers them all.
template <typename T>
struct BwdIn {
    T pi;
    V3<T> m, B, v, uk, lam, lacc, yprev;
    double g0;
    uint8_t p1, p2;
};

template <typename T>
__device__ __forceinline__ BwdIn<T> load_bwd(const StageBwdArgs<T>& a, int N, int i, bool seed) {
    BwdIn<T> d;
    const V3<T> z = v3<T>(0, 0, 0);
    d.m = d.B = d.v = d.uk = d.lacc = d.yprev = z;
    d.g0 = 0.0;
    d.p1 = d.p2 = 0;
    d.pi = gat(a.psi, i);
    d.lam = ld3u(a.lamp, N, i);
    if (!seed) {
        d.m = ld3u(a.ys, N, i);
        d.B = ld3u(a.Bs, N, i);
        d.v = ld3u(a.ell, N, i);
        d.uk = ld3u(a.u_cur, N, i);
        d.g0 = gat(a.gpsi, i);
        if (a.stage < 3 && a.lacc_in) d.lacc = ld3u(a.lacc_in, N, i);
        if (a.stage == 0 && a.port1) {
            d.p1 = gat(a.port1, i);
            d.p2 = gat(a.port2, i);
        }
    }
    if (a.y_prev) d.yprev = ld3u(a.y_prev, N, i);
    return d;
}

template <typename T, int MR, bool LIN = false>
__global__ void __launch_bounds__(512) k_stage_bwd(const BatchArgs<T> ba, const BwdL L) {
    using C = cplx<T>;
    constexpr int NV = 7;  // u_x, u_y, u_z, psi, m_x, m_y, m_z (stage state y_s)
    const int nvu = L.stage_m ? 7 : 4;  // without room in LDS, y_s neighbours come from global memory
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int2 wk = ba.single ? make_int2(0, (int)blockIdx.x) : ba.work[blockIdx.x];
    const KParams<T> p = ba.ptab[wk.x];
    const InstTab& tb = ba.itab[wk.x];
    const StageBwdArgs<T> a = resolve_bwd<T>(p, tb, L);
    const cplx<T>* __restrict__ twx = role<cplx<T>>(tb, B_TWX);
    const int Px = p.Px, nx = p.nx, N = p.N;
    const bool seed = a.stage < 0;
    const bool demag_in = a.do_inv && !seed, demag_any = (a.do_inv | a.do_fwd) != 0;
    const LocalSmem<T> LS = local_smem<T>(smem_raw, Px, demag_any);
    C* Z = LS.Z;
    T* R = LS.R;
    const int r0 = 2 * wk.y;
    const bool v1 = r0 + 1 < p.nrows;
    const SigMap sm{0, ilog2_rt(Px)};
    // work items are (row, x) pairs of the two rows, item = rr * nx + x; the
    // inputs of this thread's first item are requested before the staging
    // (in float; the float64 inputs would not fit the registers across the FFT)
    const int nitem = v1 ? 2 * nx : nx;
    constexpr bool kPre = sizeof(T) == 4;
    BwdIn<T> pre;
    if (kPre && (int)threadIdx.x < nitem) pre = load_bwd(a, N, r0 * nx + threadIdx.x, seed);

    {
        const T* const src[NV] = {a.u_cur, a.u_cur, a.u_cur, a.psi, a.ys, a.ys, a.ys};
        const int comp[NV] = {0, 1, 2, 0, 0, 1, 2};
        stage_inputs<T, NV, true>(p, r0, v1, !seed && (p.terms & 1), nvu, src, comp, R, demag_in ? a.S : nullptr, Z,
                            demag_any ? twx : nullptr, LS.Tw);
    }
    __syncthreads();
    if (demag_in) fft_lds<C, true, MR>(Z, sm, Px, 3, LS.Tw);

    const T dt = p.dt;
    // l_{s-1} = cl lambda' + cm mu_s (0-based stages): RK4 weights b = (1,2,2,1)/6 and nodes c = (0,1/2,1/2,1)
    const T cl = (a.stage == 1) ? dt / (T)6 : dt / (T)3;
    const T cm = (a.stage == 3) ? dt : dt / (T)2;

    const int iy0 = r0 % p.ny, iz0 = r0 / p.ny;
    for (int it = threadIdx.x; it < nitem; it += blockDim.x) {
        {
            const int rr = it >= nx ? 1 : 0;
            const int x = it - rr * nx;
            const int r = r0 + rr;
            const int q = rr + 1;
            int iy = iy0 + rr, iz = iz0;
            if (iy == p.ny) iy = 0, iz += 1;
            const int i = r * nx + x;
            const BwdIn<T> d = (kPre && it == (int)threadIdx.x) ? pre : load_bwd(a, N, i, seed);
            const T pi = d.pi;
            V3<T> un = v3<T>(0, 0, 0);
            if (seed) {
                V3<T> ell = a.seed_unit ? d.lam : (dt / (T)6) * d.lam;
                if constexpr (LIN) {
                    // the same fused multiply-adds, in the same order, as the stage-sum kernel from zero
                    ell = v3<T>(0, 0, 0);
                    for (int j = 0; j < L.lin_nt; ++j) {
                        const V3<T> sj = ld3(static_cast<const T*>(L.lin_src[j]), N, i);
                        const T c = (T)L.lin_c[j];
                        ell = v3<T>(fma(c, sj.x, ell.x), fma(c, sj.y, ell.y), fma(c, sj.z, ell.z));
                    }
                }
                st3u(a.ell, N, i, ell);
                un = field_adjoint(p, ell, d.yprev, x, iy, iz, pi);
                st3u(a.u_next, N, i, un);
            } else {
                const V3<T> m = d.m;
                const V3<T> B = d.B;
                const V3<T> v = d.v;
                const V3<T> uk = d.uk;
                V3<T> mu = v3<T>(0, 0, 0);
                if (pi > p.psi_freeze) {
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
                        return v3<T>(R[(qq * nvu + 0) * nx + xx], R[(qq * nvu + 1) * nx + xx], R[(qq * nvu + 2) * nx + xx]);
                    };
                    auto RP = [&](int qq, int xx) { return R[(qq * nvu + 3) * nx + xx]; };
                    auto RM = [&](int qq, int xx) {
                        if (nvu < 7) return ld3(a.ys, N, (r0 - 1 + qq) * nx + xx);
                        return v3<T>(R[(qq * nvu + 4) * nx + xx], R[(qq * nvu + 5) * nx + xx], R[(qq * nvu + 6) * nx + xx]);
                    };
                    auto nb = [&](V3<T> uj, T pj, V3<T> mj, T w) {
                        const T s = pi + pj;
                        if (s != (T)0) {
                            const T is = recip(s);
                            mu = mu + (w * pi * is) * uj - (w * pj * is) * uk;
                            g -= (double)(w * pj * is * is) * (double)dot(uk + uj, mj - m);
                        }
                    };
                    if (x > 0) nb(RU(q, x - 1), RP(q, x - 1), RM(q, x - 1), p.exw[0]);
                    if (x < nx - 1) nb(RU(q, x + 1), RP(q, x + 1), RM(q, x + 1), p.exw[0]);
                    if (iy > 0) nb(RU(q - 1, x), RP(q - 1, x), RM(q - 1, x), p.exw[1]);
                    if (iy < p.ny - 1) nb(RU(q + 1, x), RP(q + 1, x), RM(q + 1, x), p.exw[1]);
                    const int sl = nx * p.ny;
                    if (iz > 0) nb(ld3(a.u_cur, N, i - sl), glb(a.psi)[i - sl], ld3(a.ys, N, i - sl), p.exw[2]);
                    if (iz < p.nz - 1) nb(ld3(a.u_cur, N, i + sl), glb(a.psi)[i + sl], ld3(a.ys, N, i + sl), p.exw[2]);
                }
                if (demag_in) {
                    const C z01 = Z[lp(x) + lp(rr * Px)];
                    const C z2 = Z[lp(x) + lp(2 * Px)];
                    const V3<T> cu = v3<T>(z01.x, z01.y, rr == 0 ? z2.x : z2.y);
                    mu = mu + pi * cu;
                    g += (double)dot(m, cu);
                }
                if (p.terms & 8) {
                    const V3<T> ua = v3<T>(p.u[0], p.u[1], p.u[2]);
                    mu = mu + (p.anis * dot(uk, ua)) * ua;
                }
                // curve objective at stage 0: its explicit psi dependence, dJ/dpsi_i += c_n m_x,i - c_n M(n)
                if (a.port1 && a.src_lin == 2) g += (double)a.src1 * (double)m.x - (double)a.src2;
                gput(a.gpsi, i, d.g0 + g);
                const V3<T> lsum = (a.stage == 3 ? d.lam : d.lacc) + mu;
                if (a.stage > 0) {
                    st3u(a.lacc_out, N, i, lsum);
                    const V3<T> ell = cl * d.lam + cm * mu;
                    st3u(a.ell, N, i, ell);
                    un = field_adjoint(p, ell, d.yprev, x, iy, iz, pi);
                    st3u(a.u_next, N, i, un);
                } else {
                    V3<T> lam = lsum;
                    if (a.port1 && a.src_lin == 2) {
                        lam.x = lam.x + a.src1 * pi;  // curve objective: dJ/dm_x,i = c_n psi_i
                    } else if (a.port1) {
                        // source dJ/dm_n of the port objective (y component)
                        const T src = (d.p1 ? a.src1 : (T)0) + (d.p2 ? a.src2 : (T)0);
                        lam.y = lam.y + (a.src_lin ? src : src * m.y);
                    }
                    st3u(a.lacc_out, N, i, lam);
                    if (a.y_prev) {
                        const V3<T> ell = (dt / (T)6) * lam;
                        st3u(a.ell, N, i, ell);
                        un = field_adjoint(p, ell, d.yprev, x, iy, iz, pi);
                        st3u(a.u_next, N, i, un);
                    }
                }
            }
            if (a.do_fwd) {
                T* zr = reinterpret_cast<T*>(Z);
                Z[lp(x) + lp(rr * Px)] = cmk<C>(un.x, un.y);
                zr[2 * (lp(x) + lp(2 * Px)) + rr] = un.z;
                if (!v1) {
                    Z[lp(x) + lp(Px)] = cmk<C>(0, 0);
                    zr[2 * (lp(x) + lp(2 * Px)) + 1] = (T)0;
                }
            }
        }
    }
    if (a.do_fwd) {
        for (int x = nx + threadIdx.x; x < Px; x += blockDim.x) {
            Z[lp(x)] = cmk<C>(0, 0);
            Z[lp(x) + lp(Px)] = cmk<C>(0, 0);
            Z[lp(x) + lp(2 * Px)] = cmk<C>(0, 0);
        }
        __syncthreads();
        fft_lds<C, false, MR>(Z, sm, Px, 3, LS.Tw);
        pack_lds_to_rows(p, a.S, r0, v1, Z);
    }
}

// ---------------------------------------------------------------------------
// column kernel of a single-layer grid (nz = 1): the first and the last pass of
// the y transforms work on global memory directly
// ---------------------------------------------------------------------------
// The y transform of length L = Py = 2^lL starts with a pass of radix
// R1 = 2^min(log2 MR, lL) and the inverse ends with one; the passes in between
// are those of fft_lds, so the factorisation depends only on (L, MR) and every
// tiling computes the same bits.
//  - The first forward pass (no twiddles) reads its inputs from the x-spectrum
//    in global memory: its inputs j + r L/R1 with r >= R1/2 lie at rows
//    >= L/2 >= ny, the zero padding, and are not read.
//  - The last inverse pass writes the rows y < ny straight to global memory;
//    its outputs with r >= R1/2 lie in the padding and are not stored.
// Against staging the columns in LDS and copying them out this saves one LDS
// round trip and one barrier at each end.
//
// The x-spectrum columns of bins 0 and Kx - 1 = Px/2 are real (the x DFT of
// real rows at those bins), so one block transforms both as one complex column
// P = X(0) + i X(Px/2).  After the forward y transform the two parts separate
// by their Hermitian symmetry, A(ky) = (P(ky) + conj P(-ky)) / 2 and
// B(ky) = (P(ky) - conj P(-ky)) / 2i; each is multiplied by its own bin's
// tensor spectrum, and Q = A' + i B' (rebuilt for -ky from the symmetry of the
// real results) is transformed back: its real part is the field column of bin
// 0, its imaginary part that of bin Px/2.  An instance packs (p.pack) where
// bin Px/2 is the only bin of the last spectrum tile (Kx > TW) and the launch
// is large; that tile then needs no block of its own, and a launch of Kx
// columns becomes one of Kx - 1, a multiple of the CU count on the large grids.

// Stockham passes from lNs = lb to lNs = le, largest radix first (as fft_lds).
template <typename C, bool INV, int MAXREG>
__device__ __forceinline__ void fft_lds_range(C* buf, const SigMap sm, int lL, int lb, int le, int nsig,
                                              const C* __restrict__ tw) {
    int lNs = lb;
    while (lNs < le) {
        const int rem = le - lNs;
        if constexpr (MAXREG >= 16) {
            if (rem >= 4) {
                fft_pass<C, INV, 16, MAXREG>(buf, sm, lL, lNs, nsig, tw);
                lNs += 4;
                continue;
            }
        }
        if constexpr (MAXREG >= 8) {
            if (rem >= 3) {
                fft_pass<C, INV, 8, MAXREG>(buf, sm, lL, lNs, nsig, tw);
                lNs += 3;
                continue;
            }
        }
        if (rem >= 2) {
            fft_pass<C, INV, 4, MAXREG>(buf, sm, lL, lNs, nsig, tw);
            lNs += 2;
        } else {
            fft_pass<C, INV, 2, MAXREG>(buf, sm, lL, lNs, nsig, tw);
            lNs += 1;
        }
    }
}

// F1: radix-R1 first forward pass from global memory into LDS.  Work item
// (component c, bin tk, j): inputs at rows j + r L/R1, r < R1/2 (rows >= ny
// read as zero), outputs to positions j R1 + r.
// Sk1: bin Px/2 of row 0, component 0, where bin tk = 0 is the packed pair (else null).
template <typename C, int R1>
__device__ __forceinline__ void col2d_first(C* Z, const C* __restrict__ Sk, const C* __restrict__ Sk1, size_t cs,
                                            int ltk, int lL, int ny) {
    constexpr int LR = ilog2(R1);
    constexpr unsigned rb = 128;  // one row of a spectrum tile
    const unsigned cb = (unsigned)(cs * sizeof(C));
    const int lnb = lL - LR;
    const int total = 3 << (ltk + lnb);
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int tk = it & ((1 << ltk) - 1);
        const int j = (it >> ltk) & ((1 << lnb) - 1);
        const int c = it >> (ltk + lnb);
        // byte offsets from the block's base: component c, row y, bin tk (all below 2^32)
        const unsigned ob = (unsigned)c * cb + (unsigned)tk * (unsigned)sizeof(C);
        C v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int y = j + (r << lnb);
            v[r] = (r < R1 / 2 && y < ny) ? gldc_at(Sk, ob + (unsigned)y * rb) : cmk<C>(0, 0);
        }
        if (Sk1 != nullptr && tk == 0) {
            // the packed pair: imaginary part from bin Px/2 (its real column)
#pragma unroll
            for (int r = 0; r < R1 / 2; ++r) {
                const int y = j + (r << lnb);
                if (y < ny) v[r].y = gldc_at(Sk1, (unsigned)c * cb + (unsigned)y * rb).x;
            }
        }
        dft_half_in<C, false, R1>(v);
        // the point offset r 2^ltk shares no bit with the base, so the pad splits (as in fft_pass)
        C* pz = Z + lp((c << (lL + ltk)) + ((j << LR) << ltk) + tk);
#pragma unroll
        for (int r = 0; r < R1; ++r) pz[lp(r << ltk)] = v[r];
    }
    __syncthreads();
}

// Last inverse pass (radix R1, Ns = L/R1) from LDS straight to global memory:
// outputs at rows j + r L/R1 for r < R1/2 and rows < ny.
template <typename C, int R1>
__device__ __forceinline__ void col2d_last(const C* Z, C* __restrict__ Sw, C* __restrict__ Sw1, size_t cs, int ltk,
                                           int lL, int ny, int kvalid, const C* __restrict__ tw) {
    constexpr int LR = ilog2(R1);
    constexpr unsigned rb = 128;  // one row of a spectrum tile
    const unsigned cb = (unsigned)(cs * sizeof(C));
    const int lnb = lL - LR;
    const int total = 3 << (ltk + lnb);
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int tk = it & ((1 << ltk) - 1);
        const int j = (it >> ltk) & ((1 << lnb) - 1);
        const int c = it >> (ltk + lnb);
        C v[R1];
        const C* pz = Z + lp((c << (lL + ltk)) + (j << ltk) + tk);
        const int ks = lnb + ltk;
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = pz[lp(r << ks)];
        // twiddles of the last pass: index r * j (Ns = L / R1, so jm = j)
#pragma unroll
        for (int r = 1; r < R1; ++r) v[r] = cmul(v[r], cconj(tw[r * j]));
        dft_half_out<C, true, R1>(v);
        if (Sw1 != nullptr && tk == 0) {
            // the packed pair: real part to bin 0, imaginary part to bin Px/2
#pragma unroll
            for (int r = 0; r < R1 / 2; ++r) {
                const int y = j + (r << lnb);
                if (y < ny) {
                    const unsigned o = (unsigned)c * cb + (unsigned)y * rb;
                    gstc_at(Sw, o, cmk<C>(v[r].x, 0));
                    gstc_at(Sw1, o, cmk<C>(v[r].y, 0));
                }
            }
        } else if (tk < kvalid) {
            const unsigned ob = (unsigned)c * cb + (unsigned)tk * (unsigned)sizeof(C);
#pragma unroll
            for (int r = 0; r < R1 / 2; ++r) {
                const int y = j + (r << lnb);
                if (y < ny) gstc_at(Sw, ob + (unsigned)y * rb, v[r]);
            }
        }
    }
}

// Tensor multiply of the packed pair of bins 0 and Px/2 (bin tk = 0 of its
// block): one work item per (ky, -ky), ky <= Py/2.  Nk1: bin Px/2's tensor.
template <typename T>
__device__ __forceinline__ void col2d_mul_pair(cplx<T>* Z, int TK, int plane, int Py, const T* Nt,
                                               const T* __restrict__ Nk, const T* __restrict__ Nk1, int nt_lds,
                                               int Ky2) {
    using C = cplx<T>;
    constexpr int TW = spec_tile<T>();
    const int cstr = Ky2 * TK;
    const size_t gstr = (size_t)Ky2 * TW;
    const int pp = lp(plane), pp2 = lp(2 * plane);  // lp(c plane + e) = lp(e) + lp(c plane), e < plane
    for (int ky = threadIdx.x; ky <= Py / 2; ky += blockDim.x) {
        auto NT = [&](int comp) -> T { return nt_lds ? Nt[comp * cstr + ky * TK] : glb(Nk)[comp * gstr + (size_t)ky * TW]; };
        auto NT1 = [&](int comp) -> T { return glb(Nk1)[comp * gstr + (size_t)ky * TW]; };
        const T axx = NT(0), ayy = NT(1), azz = NT(2), axy = NT(3);
        const T bxx = NT1(0), byy = NT1(1), bzz = NT1(2), bxy = NT1(3);
        const int e = ky * TK, em = ((Py - ky) & (Py - 1)) * TK;
        C* const ze = Z + lp(e);
        const C u0 = ze[0], u1 = ze[pp], u2 = ze[pp2];
        if (em == e) {
            // ky = 0 or Py/2: both parts are real, A = Re P and B = Im P
            ze[0] = cmk<C>(axx * u0.x + axy * u1.x, bxx * u0.y + bxy * u1.y);
            ze[pp] = cmk<C>(axy * u0.x + ayy * u1.x, bxy * u0.y + byy * u1.y);
            ze[pp2] = cmk<C>(azz * u2.x, bzz * u2.y);
            continue;
        }
        C* const zm = Z + lp(em);
        const C v0 = zm[0], v1 = zm[pp], v2 = zm[pp2];
        const T h = (T)0.5;
        // A = (u + conj v) / 2, B = (u - conj v) / 2i
        const C A0 = cmk<C>(h * (u0.x + v0.x), h * (u0.y - v0.y)), B0 = cmk<C>(h * (u0.y + v0.y), h * (v0.x - u0.x));
        const C A1 = cmk<C>(h * (u1.x + v1.x), h * (u1.y - v1.y)), B1 = cmk<C>(h * (u1.y + v1.y), h * (v1.x - u1.x));
        const C A2 = cmk<C>(h * (u2.x + v2.x), h * (u2.y - v2.y)), B2 = cmk<C>(h * (u2.y + v2.y), h * (v2.x - u2.x));
        const C qa0 = cmk<C>(axx * A0.x + axy * A1.x, axx * A0.y + axy * A1.y);
        const C qa1 = cmk<C>(axy * A0.x + ayy * A1.x, axy * A0.y + ayy * A1.y);
        const C qa2 = cmk<C>(azz * A2.x, azz * A2.y);
        const C qb0 = cmk<C>(bxx * B0.x + bxy * B1.x, bxx * B0.y + bxy * B1.y);
        const C qb1 = cmk<C>(bxy * B0.x + byy * B1.x, bxy * B0.y + byy * B1.y);
        const C qb2 = cmk<C>(bzz * B2.x, bzz * B2.y);
        // Q(ky) = A' + i B', Q(-ky) = conj A' + i conj B'
        ze[0] = cmk<C>(qa0.x - qb0.y, qa0.y + qb0.x);
        ze[pp] = cmk<C>(qa1.x - qb1.y, qa1.y + qb1.x);
        ze[pp2] = cmk<C>(qa2.x - qb2.y, qa2.y + qb2.x);
        zm[0] = cmk<C>(qa0.x + qb0.y, qb0.x - qa0.y);
        zm[pp] = cmk<C>(qa1.x + qb1.y, qb1.x - qa1.y);
        zm[pp2] = cmk<C>(qa2.x + qb2.y, qb2.x - qa2.y);
    }
}

// Tensor multiply of the transformed columns in place, one work item per
// (ky, x-bin) with the three components (2D tensor: xx, yy, zz, xy; xy odd in ky).
// Nk1: tensor spectrum of bin Px/2 where bin tk = 0 is the packed pair (else null).
template <typename T>
__device__ __forceinline__ void col2d_mul(cplx<T>* Z, int TK, int ltk, int plane, int Py, int k0, int Kx, const T* Nt,
                                          const T* __restrict__ Nk, const T* __restrict__ Nk1, int nt_lds, int Ky2) {
    using C = cplx<T>;
    constexpr int TW = spec_tile<T>();
    const int total = Py << ltk;
    const int tk0 = Nk1 != nullptr ? 1 : 0;  // the packed pair's bin is done apart
    const int pp = lp(plane), pp2 = lp(2 * plane);
    // tensor component comp of row kyr: from the LDS tile, or from memory at an
    // unsigned 32-bit offset from the block's base (a scalar-base load)
    auto body = [&](auto lds_c) {
        constexpr bool LDS = decltype(lds_c)::value;
        const unsigned cstr = LDS ? (unsigned)(Ky2 * TK) : (unsigned)(Ky2 * TW);
        const T* __restrict__ nb = LDS ? Nt : Nk;
        for (int it = threadIdx.x; it < total; it += blockDim.x) {
            const int tk = it & (TK - 1);
            const int ky = it >> ltk;
            if (k0 + tk >= Kx || tk < tk0) continue;
            const bool fy = ky > Py / 2;
            const int kyr = fy ? Py - ky : ky;
            const unsigned o = LDS ? (unsigned)((kyr << ltk) + tk) : (unsigned)(kyr * TW + tk);
            auto NT = [&](int comp) -> T {
                if constexpr (LDS) return nb[comp * cstr + o];
                else return gld_at(nb, (comp * cstr + o) * (unsigned)sizeof(T));
            };
            const T nxx = NT(0), nyy = NT(1), nzz = NT(2);
            const T nxy = fy ? -NT(3) : NT(3);
            // e < plane, a power of two: lp(c plane + e) = lp(e) + lp(c plane)
            C* const ze = Z + lp((ky << ltk) + tk);
            const C a = ze[0], b = ze[pp], z = ze[pp2];
            ze[0] = cmk<C>(nxx * a.x + nxy * b.x, nxx * a.y + nxy * b.y);
            ze[pp] = cmk<C>(nxy * a.x + nyy * b.x, nxy * a.y + nyy * b.y);
            ze[pp2] = cmk<C>(nzz * z.x, nzz * z.y);
        }
    };
    if (nt_lds)
        body(std::integral_constant<bool, true>());
    else
        body(std::integral_constant<bool, false>());
    if (Nk1 != nullptr) col2d_mul_pair<T>(Z, TK, plane, Py, Nt, Nk, Nk1, nt_lds, Ky2);
    __syncthreads();
}

// The whole column computation of one block for a single-layer instance.
template <typename T, int MR>
__device__ __forceinline__ void col2d_body(const KParams<T>& p, const InstTab& tb, int k0, int TK, int sid, int nt_lds,
                                           unsigned char* smem_raw) {
    using C = cplx<T>;
    C* __restrict__ S = role<C>(tb, sid);
    const T* __restrict__ nhat = role<T>(tb, B_NHAT);
    const C* __restrict__ twy = role<C>(tb, B_TWY);
    const int Py = p.Py, ny = p.ny;
    constexpr int TW = spec_tile<T>();
    const int kt = k0 / TW, ko = k0 % TW;
    const size_t cs = (size_t)p.ktiles * p.nrows * TW;
    C* __restrict__ Sk = S + (size_t)kt * p.nrows * TW + ko;  // bin k0 of row 0, component 0
    const int NR = p.ncomp * p.Kz2 * p.Ky2;
    const T* __restrict__ Nk = nhat + (size_t)kt * NR * TW + ko;
    // bins 0 and Px/2 as one complex column (block of bin 0, where Px/2 is alone in the last tile)
    const bool pk = k0 == 0 && p.pack;
    C* __restrict__ Sk1 = pk ? S + (size_t)((p.Kx - 1) / TW) * p.nrows * TW : nullptr;
    const T* __restrict__ Nk1 = pk ? nhat + (size_t)((p.Kx - 1) / TW) * NR * TW : nullptr;
    if (Py == 1) {
        // a single row: no y transform, the multiply alone (ky = 0); the packed
        // block also multiplies bin Px/2 (item tk = TK)
        for (int tk = threadIdx.x; tk < TK + (pk ? 1 : 0); tk += blockDim.x) {
            if (tk < TK && k0 + tk >= p.Kx) continue;
            C* const sk = tk < TK ? Sk + tk : Sk1;
            const auto N = glb(tk < TK ? Nk + tk : Nk1);
            const T nxx = N[0], nyy = N[TW], nzz = N[2 * TW], nxy = N[3 * TW];
            const C a = gld(sk), b = gld(sk + cs), z = gld(sk + 2 * cs);
            gst(sk, cmk<C>(nxx * a.x + nxy * b.x, nxx * a.y + nxy * b.y));
            gst(sk + cs, cmk<C>(nxy * a.x + nyy * b.x, nxy * a.y + nyy * b.y));
            gst(sk + 2 * cs, cmk<C>(nzz * z.x, nzz * z.y));
        }
        return;
    }
    const int plane = Py * TK;
    C* Z = reinterpret_cast<C*>(smem_raw);
    C* Tw = Z + lds_pad(3 * plane);
    T* Nt = reinterpret_cast<T*>(Tw + Py);
    // the tensor-spectrum tile (when kept in LDS) and the twiddles
    constexpr int RPU = 16 / sizeof(T);
    const int lnr = TK > RPU ? ilog2_rt(TK / RPU) : 0;
    const int rcnt = TK < RPU ? TK : RPU;
    const int ntu = nt_lds ? (p.ncomp * p.Ky2) << lnr : 0;
    struct RUnit {
        T r[RPU];
    };
    auto ltile = [&](int e) {
        RUnit u;
        const int ro = (e & ((1 << lnr) - 1)) * RPU, q = e >> lnr;
        const auto src = glb(Nk + (size_t)q * TW + ro);
        if (rcnt == RPU) {
            if constexpr (sizeof(T) == 4) {
                const vec4<float> v = *(const __attribute__((address_space(1))) vec4<float>*)src;
                u.r[0] = v.x, u.r[1] = v.y, u.r[2] = v.z, u.r[3] = v.w;
            } else {
                const vec2<double> v = *(const __attribute__((address_space(1))) vec2<double>*)src;
                u.r[0] = v.x, u.r[1] = v.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < RPU; ++k) u.r[k] = k < rcnt ? src[k] : (T)0;
        }
        return u;
    };
    auto stile = [&](int e, const RUnit& u) {
        const int ro = (e & ((1 << lnr) - 1)) * RPU, q = e >> lnr;
#pragma unroll
        for (int k = 0; k < RPU; ++k)
            if (k < rcnt) Nt[q * TK + ro + k] = u.r[k];
    };
    auto ltw = [&](int k) { return gld(twy + k); };
    auto stw = [&](int k, C w) { Tw[k] = w; };
    auto lnone = [&](int) { return 0; };
    auto snone = [&](int, int) {};
    gather3<4, 1, 1, RUnit, C, int>(ntu, ltile, stile, Py, ltw, stw, 0, lnone, snone);
    __syncthreads();

    const int lL = ilog2_rt(Py);
    const int ltk = ilog2_rt(TK);
    constexpr int LMR = ilog2(MR);
    const int lR1 = lL < LMR ? lL : LMR;
    const SigMap smy{ltk, ilog2_rt(plane)};
    // forward: the first pass from global memory, the rest in LDS
    switch (lR1) {
        case 1: col2d_first<C, 2>(Z, Sk, Sk1, cs, ltk, lL, ny); break;
        case 2: col2d_first<C, 4>(Z, Sk, Sk1, cs, ltk, lL, ny); break;
        case 3: col2d_first<C, 8>(Z, Sk, Sk1, cs, ltk, lL, ny); break;
        default:
            if constexpr (MR >= 16) col2d_first<C, 16>(Z, Sk, Sk1, cs, ltk, lL, ny);
            break;
    }
    fft_lds_range<C, false, MR>(Z, smy, lL, lR1, lL, 3 * TK, Tw);
    col2d_mul<T>(Z, TK, ltk, plane, Py, k0, p.Kx, Nt, Nk, Nk1, nt_lds, p.Ky2);
    // inverse: every pass but the last in LDS, the last to global memory
    fft_lds_range<C, true, MR>(Z, smy, lL, 0, lL - lR1, 3 * TK, Tw);
    const int kvalid = p.Kx - k0;
    switch (lR1) {
        case 1: col2d_last<C, 2>(Z, Sk, Sk1, cs, ltk, lL, ny, kvalid, Tw); break;
        case 2: col2d_last<C, 4>(Z, Sk, Sk1, cs, ltk, lL, ny, kvalid, Tw); break;
        case 3: col2d_last<C, 8>(Z, Sk, Sk1, cs, ltk, lL, ny, kvalid, Tw); break;
        default:
            if constexpr (MR >= 16) col2d_last<C, 16>(Z, Sk, Sk1, cs, ltk, lL, ny, kvalid, Tw);
            break;
    }
}

template <typename T, int MR>
__global__ void __launch_bounds__(MR >= 16 ? 512 : 768) k_col2d(const BatchArgs<T> ba, int TK, int sid, int nt_lds) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int2 wk = ba.work[blockIdx.x];  // (instance, first bin); XCD-grouped order, also for one instance
    if (wk.y >= (1 << 30)) return;      // empty item that keeps the grouping stride
    const KParams<T> p = ba.ptab[wk.x];
    col2d_body<T, MR>(p, ba.itab[wk.x], wk.y, TK, sid, nt_lds, smem_raw);
}

// ---------------------------------------------------------------------------
// column kernel: y (and z) transforms + tensor-spectrum multiply, in place
// shared memory: Z [c][z < nz][y < Py][tk] complex (padded, see lp), Tw [Py] complex,
//                Nt [comp][kz <= Pz/2][ky <= Py/2][tk] real
// ---------------------------------------------------------------------------
// Radix-16 passes need more than the 128 registers a 1024-thread block allows,
// so that variant is limited to 512 threads.
template <typename T, int NZ, int MR>
__global__ void __launch_bounds__(MR >= 16 ? 512 : (NZ >= 8 ? 1024 : 768)) k_col_conv(const BatchArgs<T> ba, int TK, int sid, int nt_lds) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int2 wk = ba.work[blockIdx.x];  // (instance, first bin); XCD-grouped order, also for one instance
    if (wk.y >= (1 << 30)) return;      // empty item that keeps the grouping stride
    const KParams<T> p = ba.ptab[wk.x];
    const InstTab& tb = ba.itab[wk.x];
    if (p.nz == 1) {
        // a single-layer instance of a batch with thicker ones: the same computation as its own handle runs
        col2d_body<T, MR>(p, tb, wk.y, TK, sid, nt_lds, smem_raw);
        return;
    }
    C* __restrict__ S = role<C>(tb, sid);
    const T* __restrict__ nhat = role<T>(tb, B_NHAT);
    const C* __restrict__ twy = role<C>(tb, B_TWY);
    const C* __restrict__ twz = role<C>(tb, B_TWZ);
    const int Kx = p.Kx, Py = p.Py, Pz = p.Pz, ny = p.ny, nz = p.nz;
    const int plane = Py * TK;
    C* Z = reinterpret_cast<C*>(smem_raw);
    C* Tw = Z + lds_pad(3 * nz * plane);
    T* Nt = reinterpret_cast<T*>(Tw + Py);
    constexpr int TW = spec_tile<T>();
    const int k0 = wk.y;  // first x-bin of the tile (TK <= TW bins inside one spectrum tile)
    const int kt = k0 / TW, ko = k0 % TW;
    const size_t cs = (size_t)p.ktiles * p.nrows * TW;
    const C* __restrict__ Sk = S + (size_t)kt * p.nrows * TW + ko;  // bin k0 of row 0, component 0
    const int NR = p.ncomp * p.Kz2 * p.Ky2;
    const T* __restrict__ Nk = nhat + (size_t)kt * NR * TW + ko;
    // bins 0 and Px/2 as one complex column (as in the single-layer kernel)
    const bool pk = k0 == 0 && p.pack;
    C* __restrict__ Sk1 = pk ? S + (size_t)((Kx - 1) / TW) * p.nrows * TW : nullptr;
    const T* __restrict__ Nk1 = pk ? nhat + (size_t)((Kx - 1) / TW) * NR * TW : nullptr;
    // The columns (zero-padded in y), the tensor-spectrum tile and the
    // twiddles, in batched chunks of 16-byte loads: the TK bins of a tile row
    // are contiguous in memory (a unit holds 2 float bins or 1 double bin; a
    // lone float bin is one 8-byte unit).  Bins past Kx inside a spectrum tile
    // are zero in memory and never stored back.
    constexpr int CPU = sizeof(T) == 4 ? 2 : 1;  // complex bins per 16-byte unit
    const int lpy = ilog2_rt(Py);
    const int lnu = TK > CPU ? ilog2_rt(TK / CPU) : 0;  // log2 units per row
    const int ucnt = TK < CPU ? TK : CPU;                // bins per unit
    const int ncolu = (3 * nz * Py) << lnu;
    // row of S for plane cz = c * nz + z and y: component c at c * cs, row z * ny + y
    auto srow = [&](int cz, int y) {
        const int c = (cz >= nz) + (cz >= 2 * nz);
        return (size_t)c * cs + (size_t)((cz - c * nz) * ny + y) * TW;
    };
    struct Unit {
        C c[CPU];
    };
    auto lcol = [&](int e) {
        Unit u;
        const int uo = (e & ((1 << lnu) - 1)) * CPU;
        const int row = e >> lnu;
        const int y = row & (Py - 1), cz = row >> lpy;
#pragma unroll
        for (int k = 0; k < CPU; ++k) u.c[k] = cmk<C>(0, 0);
        if (y < ny) {
            const C* src = Sk + srow(cz, y) + uo;
            if constexpr (CPU == 2) {
                if (ucnt == 2) {
                    const vec4<float> q = *(const __attribute__((address_space(1))) vec4<float>*)src;
                    u.c[0] = cmk<C>(q.x, q.y);
                    u.c[1] = cmk<C>(q.z, q.w);
                } else {
                    u.c[0] = gld(src);
                }
            } else {
                u.c[0] = gld(src);
            }
            if (pk && uo == 0) u.c[0].y = gld(Sk1 + srow(cz, y)).x;
        }
        return u;
    };
    auto scol = [&](int e, const Unit& u) {
        const int uo = (e & ((1 << lnu) - 1)) * CPU;
        const int row = e >> lnu;
        const int base = row * TK + uo;  // (cz * Py + y) * TK + bin
#pragma unroll
        for (int k = 0; k < CPU; ++k)
            if (k < ucnt) Z[lp(base + k)] = u.c[k];
    };
    // tensor-spectrum tile: TK reals per row q = (comp * Kz2 + kz) * Ky2 + ky, 16-byte units
    constexpr int RPU = 16 / sizeof(T);  // reals per unit
    const int lnr = TK > RPU ? ilog2_rt(TK / RPU) : 0;
    const int rcnt = TK < RPU ? TK : RPU;
    const int ntu = nt_lds ? (p.ncomp * p.Kz2 * p.Ky2) << lnr : 0;
    struct RUnit {
        T r[RPU];
    };
    auto ltile = [&](int e) {
        RUnit u;
        const int ro = (e & ((1 << lnr) - 1)) * RPU, q = e >> lnr;
        const auto src = glb(Nk + (size_t)q * TW + ro);
        if (rcnt == RPU) {
            if constexpr (sizeof(T) == 4) {
                const vec4<float> v = *(const __attribute__((address_space(1))) vec4<float>*)src;
                u.r[0] = v.x, u.r[1] = v.y, u.r[2] = v.z, u.r[3] = v.w;
            } else {
                const vec2<double> v = *(const __attribute__((address_space(1))) vec2<double>*)src;
                u.r[0] = v.x, u.r[1] = v.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < RPU; ++k) u.r[k] = k < rcnt ? src[k] : (T)0;
        }
        return u;
    };
    auto stile = [&](int e, const RUnit& u) {
        const int ro = (e & ((1 << lnr) - 1)) * RPU, q = e >> lnr;
#pragma unroll
        for (int k = 0; k < RPU; ++k)
            if (k < rcnt) Nt[q * TK + ro + k] = u.r[k];
    };
    auto ltw = [&](int k) { return gld(twy + k); };
    auto stw = [&](int k, C w) { Tw[k] = w; };
    gather3<4, 4, 1, Unit, RUnit, C>(ncolu, lcol, scol, ntu, ltile, stile, Py, ltw, stw);
    __syncthreads();
    const SigMap smy{ilog2_rt(TK), ilog2_rt(plane)};
    if (Py > 1) fft_lds<C, false, MR, false>(Z, smy, Py, 3 * nz * TK, Tw);
    // packed pair, 0 < ky < Py/2: A(ky) goes to position ky, B(ky) to position Py - ky
    const int hpy = Py / 2 - 1;
    if (pk && hpy > 0) {
        for (int e = threadIdx.x; e < 3 * nz * hpy; e += blockDim.x) {
            const int ky = 1 + e % hpy, cz = e / hpy;
            const int i0 = lp(cz * plane + ky * TK), i1 = lp(cz * plane + (Py - ky) * TK);
            const C u = Z[i0], v = Z[i1];
            const T h = (T)0.5;
            Z[i0] = cmk<C>(h * (u.x + v.x), h * (u.y - v.y));
            Z[i1] = cmk<C>(h * (u.y + v.y), h * (v.x - u.x));
        }
        __syncthreads();
    }

    // per (ky, tk): z transform in registers, tensor multiply, inverse z transform.
    // Packed column (tk = 0 of the packed block): positions ky < Py/2 hold A with
    // bin 0's tensor (mode 0), positions ky > Py/2 hold B(Py - ky) with bin Px/2's
    // (mode 1).  At ky = 0 and Py/2 both parts are real sequences in z: the real
    // part is transformed with bin 0's tensor (mode 2), the imaginary part with
    // bin Px/2's (mode 3), each keeping its result's real part; the two read and
    // write disjoint halves of the column, so they run as separate work items.
    const int cstr = p.Kz2 * p.Ky2 * TK;
    auto zcol = [&](const int ky, const int tk, auto mode_c) {
        constexpr int mode = decltype(mode_c)::value;
        // ky TK + tk < plane, a power of two, so lp(m plane + e) = lp(e) + m plane + (m plane) / 16
        const int ib = lp(ky * TK + tk);
        auto zoff = [&](int m) { return lp(m * plane); };
        C X[3][NZ];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                X[c][z] = z < nz ? Z[ib + zoff(c * nz + z)] : cmk<C>(0, 0);
                if constexpr (mode >= 2) X[c][z] = cmk<C>(mode == 2 ? X[c][z].x : X[c][z].y, 0);
            }
        const bool fy = mode == 0 && ky > Py / 2;
        const int kyr = ky > Py / 2 ? Py - ky : ky;
        constexpr bool use1 = mode == 1 || mode == 3;  // bin Px/2's tensor, from memory
        const T* __restrict__ Nsel = use1 ? Nk1 : Nk;
        const bool lds_t = !use1 && nt_lds;
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
                    if (z < nz) s = cadd(s, cmul(X[c][z], gld(twz + ((kz * z) & (Pz - 1)))));
                h[c] = s;
            }
            const bool fz = kz > Pz / 2;
            const int kzr = fz ? Pz - kz : kz;
            const int base = (kzr * p.Ky2 + kyr) * TK + tk;
            const size_t gbase = (size_t)(kzr * p.Ky2 + kyr) * TW + tk, gstr = (size_t)p.Kz2 * p.Ky2 * TW;
            auto NT = [&](int comp) -> T { return lds_t ? Nt[comp * cstr + base] : glb(Nsel)[comp * gstr + gbase]; };
            const T nxx = NT(0), nyy = NT(1), nzz = NT(2);
            const T nxy = fy ? -NT(3) : NT(3);
            T nxz = 0, nyz = 0;
            if (p.ncomp == 6) {
                nxz = fz ? -NT(4) : NT(4);
                nyz = NT(5);
                if (fy != fz) nyz = -nyz;
            }
            const C hx = cmk<C>(nxx * h[0].x + nxy * h[1].x + nxz * h[2].x, nxx * h[0].y + nxy * h[1].y + nxz * h[2].y);
            const C hy = cmk<C>(nxy * h[0].x + nyy * h[1].x + nyz * h[2].x, nxy * h[0].y + nyy * h[1].y + nyz * h[2].y);
            const C hz = cmk<C>(nxz * h[0].x + nyz * h[1].x + nzz * h[2].x, nxz * h[0].y + nyz * h[1].y + nzz * h[2].y);
            // inverse z DFT, only the nz planes that are kept
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                if (z >= nz) break;
                const C w = cconj(gld(twz + ((kz * z) & (Pz - 1))));
                Y[0][z] = cadd(Y[0][z], cmul(hx, w));
                Y[1][z] = cadd(Y[1][z], cmul(hy, w));
                Y[2][z] = cadd(Y[2][z], cmul(hz, w));
            }
        }
        T* const zr = reinterpret_cast<T*>(Z);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                if (z >= nz) break;
                const int i = ib + zoff(c * nz + z);
                if constexpr (mode < 2)
                    Z[i] = Y[c][z];
                else
                    zr[2 * i + (mode - 2)] = Y[c][z].x;
            }
    };
    const int npair = Py * TK;
    for (int e = threadIdx.x; e < npair; e += blockDim.x) {
        const int tk = e % TK, ky = e / TK;
        if (k0 + tk >= Kx) continue;
        if (pk && tk == 0 && (ky == 0 || 2 * ky >= Py)) continue;  // packed: below
        zcol(ky, tk, std::integral_constant<int, 0>());
    }
    if (pk) {
        // B at ky > Py/2, then the real and imaginary parts at ky = 0 and Py/2
        const int nhi = Py / 2 - 1 > 0 ? Py / 2 - 1 : 0;
        const int nself = Py > 1 ? 4 : 2;
        for (int e = threadIdx.x; e < nhi + nself; e += blockDim.x) {
            if (e < nhi) {
                zcol(Py / 2 + 1 + e, 0, std::integral_constant<int, 1>());
            } else {
                const int q = e - nhi;
                if (q & 1)
                    zcol((q >> 1) * (Py / 2), 0, std::integral_constant<int, 3>());
                else
                    zcol((q >> 1) * (Py / 2), 0, std::integral_constant<int, 2>());
            }
        }
    }
    __syncthreads();
    // packed pair: Q(ky) = A' + i B', Q(Py - ky) = conj A' + i conj B'
    if (pk && hpy > 0) {
        for (int e = threadIdx.x; e < 3 * nz * hpy; e += blockDim.x) {
            const int ky = 1 + e % hpy, cz = e / hpy;
            const int i0 = lp(cz * plane + ky * TK), i1 = lp(cz * plane + (Py - ky) * TK);
            const C a = Z[i0], b = Z[i1];
            Z[i0] = cmk<C>(a.x - b.y, a.y + b.x);
            Z[i1] = cmk<C>(a.x + b.y, b.x - a.y);
        }
        __syncthreads();
    }
    if (Py > 1) fft_lds<C, true, MR, false>(Z, smy, Py, 3 * nz * TK, Tw);
    const int ltk = ilog2_rt(TK);
    const int ncolel = 3 * nz * Py * TK;
    C* __restrict__ Sw = S + (size_t)kt * p.nrows * TW + ko;
    for (int e = threadIdx.x; e < ncolel; e += blockDim.x) {
        const int tk = e & (TK - 1);
        const int t = e >> ltk;
        const int y = t & (Py - 1), cz = t >> lpy;
        if (y < ny && k0 + tk < Kx) {
            const C v = Z[lp(e)];
            if (pk && tk == 0) {
                gst(Sw + srow(cz, y), cmk<C>(v.x, 0));
                gst(Sk1 + srow(cz, y), cmk<C>(v.y, 0));
            } else {
                gst(Sw + srow(cz, y) + tk, v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// element-wise kernels over (element, instance) grids
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_levelset(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, T a, int extrude) {
    const int inst = blockIdx.y;
    const KParams<T>& p = ptab[inst];
    const InstTab& tb = itab[inst];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const int j = extrude ? i % (p.nx * p.ny) : i;
    const T* phi = role<T>(tb, B_PHI);
    const T* pf = role<T>(tb, B_PSIF);
    const uint8_t* des = role<uint8_t>(tb, B_DES);
    role<T>(tb, B_PSI)[i] = des[i] ? (T)1 / ((T)1 + exp(-a * phi[j])) : pf[i];
}

template <typename T>
__global__ void k_levelset_vjp(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, double a,
                               int extrude) {
    const int inst = blockIdx.y;
    const KParams<T>& p = ptab[inst];
    const InstTab& tb = itab[inst];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int M = extrude ? p.nx * p.ny : p.N;
    if (j >= M) return;
    const int nl = extrude ? p.nz : 1;
    const T* phi = role<T>(tb, B_PHI);
    const double* g = role<double>(tb, B_DPSI);
    const uint8_t* des = role<uint8_t>(tb, B_DES);
    const double H = 1.0 / (1.0 + exp(-a * (double)phi[j]));
    const double hp = a * H * (1.0 - H);
    double s = 0.0;
    for (int l = 0; l < nl; ++l) {
        const int i = j + l * M;
        if (des[i]) s += hp * g[i];
    }
    role<double>(tb, B_DPHI)[j] = s;
}

template <typename T>
__global__ void k_adj_init(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, int lam_sel,
                           int use_djdm, int port, int W) {
    const int inst = blockIdx.y;
    const KParams<T>& p = ptab[inst];
    const InstTab& tb = itab[inst];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const int N = p.N;
    V3<T> l = use_djdm ? ld3(role<T>(tb, B_DJDM), N, i) : v3<T>(0, 0, 0);
    if (port == 1 && W > 0 && (p.n_p1 + p.n_p2) > 0) {
        const T s1 = p.n_p1 > 0 ? (T)(2.0 / ((double)W * p.n_p1)) : (T)0;
        const T s2 = p.n_p2 > 0 ? (T)(2.0 / ((double)W * p.n_p2)) : (T)0;
        const T src = (role<uint8_t>(tb, B_P1)[i] ? s1 : (T)0) - (role<uint8_t>(tb, B_P2)[i] ? s2 : (T)0);
        l.y = l.y + src * role<T>(tb, B_M)[N + i];
    }
    if (port == 3 && W > 0) {
        // curve objective: sources of the last window state m_N (the psi term adds to the cleared dJ/dpsi)
        const double* g = role<double>(tb, B_PSRC) + 2 * (size_t)(W - 1);
        const T pi = role<T>(tb, B_PSI)[i];
        l.x = l.x + (T)g[0] * pi;
        role<double>(tb, B_GPSI)[i] += g[0] * (double)role<T>(tb, B_M)[i] - g[1];
    }
    if (port == 2 && W > 0 && (p.n_p1 + p.n_p2) > 0) {
        // spectral objective: the stored source of the last window state m_N
        const double* g = role<double>(tb, B_PSRC) + 2 * (size_t)(W - 1);
        const T src = (role<uint8_t>(tb, B_P1)[i] ? (T)g[0] : (T)0) + (role<uint8_t>(tb, B_P2)[i] ? (T)g[1] : (T)0);
        l.y = l.y + src;
    }
    st3(role<T>(tb, lam_sel), N, i, l);
}

template <typename T>
__global__ void k_psi_grad_out(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, int use_expl) {
    const int inst = blockIdx.y;
    const KParams<T>& p = ptab[inst];
    const InstTab& tb = itab[inst];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    role<double>(tb, B_DPSI)[i] = role<double>(tb, B_GPSI)[i] + (use_expl ? role<double>(tb, B_DPSIE)[i] : 0.0);
}

// what: 0 = N doubles, 1 = 2 * nloc doubles (port partials)
template <typename T>
__global__ void k_zero(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, int sel, int what) {
    const int inst = blockIdx.y;
    const KParams<T>& p = ptab[inst];
    const int n = what == 0 ? p.N : 2 * p.nloc;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) role<double>(itab[inst], sel)[i] = 0.0;
}

// role[off * N + e] = v for e < mult * N of every instance
template <typename T>
__global__ void k_fill(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, int sel, int mult, T v,
                       int off) {
    const int inst = blockIdx.y;
    const size_t n = (size_t)mult * ptab[inst].N;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) role<T>(itab[inst], sel)[(size_t)off * ptab[inst].N + i] = v;
}

template <typename T>
__global__ void k_copy(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, int src, int src_slot,
                       int dst, int dst_slot, int mult) {
    const int inst = blockIdx.y;
    const size_t n3 = (size_t)3 * mult * ptab[inst].N;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const InstTab& tb = itab[inst];
    role<T>(tb, dst)[dst_slot * n3 + i] = role<T>(tb, src)[src_slot * n3 + i];
}

// one block per instance: J = (sum part1 / |P1| - sum part2 / |P2|) / W, fixed order
template <typename T>
__global__ void k_port_finish(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, int W) {
    __shared__ double red[2][256];
    const int inst = blockIdx.x;
    const KParams<T>& p = ptab[inst];
    const InstTab& tb = itab[inst];
    const double* part = role<double>(tb, B_PPART);
    double s1 = 0.0, s2 = 0.0;
    for (int b = threadIdx.x; b < p.nloc; b += blockDim.x) {
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
    if (threadIdx.x == 0) {
        const double i1 = p.n_p1 > 0 ? 1.0 / p.n_p1 : 0.0, i2 = p.n_p2 > 0 ? 1.0 / p.n_p2 : 0.0;
        role<double>(tb, B_SCAL)[0] = W > 0 ? (red[0][0] * i1 - red[1][0] * i2) / W : 0.0;
    }
}

// ---------------------------------------------------------------------------
// spectral port objective (Eq. 10) after a forward run
// ---------------------------------------------------------------------------

// Wave-wide sum in a fixed butterfly order (every lane receives it).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One 64-lane block per (window step n, instance): x_j(n) = sum over the
// row-pair blocks of the stored partial sums / |P_j|, in block order.
template <typename T>
__global__ __launch_bounds__(64) void k_spec_series(const KParams<T>* __restrict__ ptab,
                                                    const InstTab* __restrict__ itab) {
    const int inst = blockIdx.y, n = blockIdx.x;
    const KParams<T>& p = ptab[inst];
    const InstTab& tb = itab[inst];
    const double* part = role<double>(tb, B_PSER) + (size_t)n * 2 * p.nloc;
    double s1 = 0.0, s2 = 0.0;
    for (int b = threadIdx.x; b < p.nloc; b += 64) {
        s1 += part[2 * b];
        s2 += part[2 * b + 1];
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (threadIdx.x == 0) {
        double* x = role<double>(tb, B_SER) + 2 * (size_t)n;
        x[0] = p.n_p1 > 0 ? s1 / p.n_p1 : 0.0;
        x[1] = p.n_p2 > 0 ? s2 / p.n_p2 : 0.0;
    }
}

// t_n of window step n (state m_{n_start + 1 + n})
__device__ __forceinline__ double window_time(double t0, int64_t n_start, int n, double dt) {
    return t0 + (double)(n_start + 1 + n) * dt;
}

// One block per (sample frequency q, instance): C_jq = 1/W sum_n x_j(n)
// cos(2 pi f_q t_n), S_jq likewise with sin; fixed-order reduction.
template <typename T>
__global__ __launch_bounds__(256) void k_spec_dft(const KParams<T>* __restrict__ ptab,
                                                  const InstTab* __restrict__ itab, const double* __restrict__ fc,
                                                  int W, double t0, int64_t n_start, double dt) {
    __shared__ double red[4][4];
    const int inst = blockIdx.y, q = blockIdx.x;
    const InstTab& tb = itab[inst];
    const double* x = role<double>(tb, B_SER);
    const double w = 6.283185307179586476925286766559 * fc[q];
    double c1 = 0.0, s1 = 0.0, c2 = 0.0, s2 = 0.0;
    for (int n = threadIdx.x; n < W; n += 256) {
        double sn, cn;
        sincos(w * window_time(t0, n_start, n, dt), &sn, &cn);
        c1 += x[2 * n] * cn;
        s1 += x[2 * n] * sn;
        c2 += x[2 * n + 1] * cn;
        s2 += x[2 * n + 1] * sn;
    }
    c1 = wave_sum(c1);
    s1 = wave_sum(s1);
    c2 = wave_sum(c2);
    s2 = wave_sum(s2);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = c1;
        red[1][wv] = s1;
        red[2][wv] = c2;
        red[3][wv] = s2;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        const double v = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
        role<double>(tb, B_SPC)[4 * (size_t)q + k] = v / W;
    }
}

// |X| of one (C, S) pair
__device__ __forceinline__ double spec_mag(double c, double s) { return sqrt(c * c + s * s); }

// One block per instance: J = sum_q c_1q |X_1q| + c_2q |X_2q|, in q order.
template <typename T>
__global__ void k_spec_finish(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab,
                              const double* __restrict__ fc, int K) {
    const InstTab& tb = itab[blockIdx.x];
    if (threadIdx.x != 0) return;
    const double* X = role<double>(tb, B_SPC);
    double J = 0.0;
    for (int q = 0; q < K; ++q)
        J += fc[K + q] * spec_mag(X[4 * q], X[4 * q + 1]) + fc[2 * K + q] * spec_mag(X[4 * q + 2], X[4 * q + 3]);
    role<double>(tb, B_SCAL)[0] = J;
}

// Per window step n: g_j(n) = sum_q c_jq (C_jq cos + S_jq sin)(2 pi f_q t_n) /
// (W |X_jq|), divided by |P_j| (the source of each node of port j).  A
// sample frequency with |X| = 0 (the magnitude's kink) contributes nothing.
template <typename T>
__global__ __launch_bounds__(256) void k_spec_src(const KParams<T>* __restrict__ ptab,
                                                  const InstTab* __restrict__ itab, const double* __restrict__ fc,
                                                  int K, int W, double t0, int64_t n_start, double dt) {
    const int inst = blockIdx.y;
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= W) return;
    const KParams<T>& p = ptab[inst];
    const InstTab& tb = itab[inst];
    const double* X = role<double>(tb, B_SPC);
    const double t = window_time(t0, n_start, n, dt);
    double g1 = 0.0, g2 = 0.0;
    for (int q = 0; q < K; ++q) {
        double sn, cn;
        sincos(6.283185307179586476925286766559 * fc[q] * t, &sn, &cn);
        const double a1 = spec_mag(X[4 * q], X[4 * q + 1]), a2 = spec_mag(X[4 * q + 2], X[4 * q + 3]);
        if (a1 > 0.0) g1 += fc[K + q] * (X[4 * q] * cn + X[4 * q + 1] * sn) / a1;
        if (a2 > 0.0) g2 += fc[2 * K + q] * (X[4 * q + 2] * cn + X[4 * q + 3] * sn) / a2;
    }
    double* out = role<double>(tb, B_PSRC) + 2 * (size_t)n;
    out[0] = p.n_p1 > 0 ? g1 / ((double)W * p.n_p1) : 0.0;
    out[1] = p.n_p2 > 0 ? g2 / ((double)W * p.n_p2) : 0.0;
}

// Curve objective (Eq. 8): per window step n, the particle average
// M(n) = sum psi m_x / sum psi from the row-pair blocks' stored sums (block
// order; M = 0 without material) and the sources c_n = weight_n sign(M(n) -
// target_n) / sum psi and c_n M(n): dJ/dm_x,i(n) = c_n psi_i and
// dJ/dpsi_i += c_n m_x,i(n) - c_n M(n).  grid (ceil(W / 256), instances).
template <typename T>
__global__ __launch_bounds__(256) void k_curve_series(const KParams<T>* __restrict__ ptab,
                                                      const InstTab* __restrict__ itab,
                                                      const double* __restrict__ tw, int W) {
    const int inst = blockIdx.y;
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= W) return;
    const KParams<T>& p = ptab[inst];
    const InstTab& tb = itab[inst];
    const double* part = role<double>(tb, B_PSER) + (size_t)n * 2 * p.nloc;
    double s = 0.0, S = 0.0;
    for (int b = 0; b < p.nloc; ++b) {
        s += part[2 * b];
        S += part[2 * b + 1];
    }
    const double M = S != 0.0 ? s / S : 0.0;
    const double d = M - tw[n];
    role<double>(tb, B_SER)[2 * (size_t)n] = M;
    double* g = role<double>(tb, B_PSRC) + 2 * (size_t)n;
    const double c = S != 0.0 ? tw[W + n] * (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / S : 0.0;
    g[0] = c;
    g[1] = c * M;
}

// One block per instance: J = sum_n weight_n |M(n) - target_n|, fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_curve_finish(const KParams<T>* __restrict__ ptab,
                                                      const InstTab* __restrict__ itab,
                                                      const double* __restrict__ tw, int W) {
    __shared__ double red[4];
    const InstTab& tb = itab[blockIdx.x];
    const double* M = role<double>(tb, B_SER);
    double s = 0.0;
    for (int n = threadIdx.x; n < W; n += 256) s += tw[W + n] * fabs(M[2 * n] - tw[n]);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) role<double>(tb, B_SCAL)[0] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Explicit Runge-Kutta helpers of the adaptive integrator: stage sums and the
// max-norm of the embedded error estimate.
template <typename T>
__global__ __launch_bounds__(256) void k_lincomb(int n, T* __restrict__ out, const T* __restrict__ base,
                                                 LinTerms<T> lt) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    T v = base ? base[e] : (T)0;
    for (int j = 0; j < lt.nt; ++j) v = fma((T)lt.c[j], lt.src[j][e], v);
    out[e] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_err_norm(int n, const T* __restrict__ y, const T* __restrict__ y5,
                                                  LinTerms<T> lt, double rtol, double atol,
                                                  double* __restrict__ part) {
    __shared__ double red[4];
    const int e = blockIdx.x * 256 + threadIdx.x;
    double r = 0.0;
    if (e < n) {
        T v = (T)0;
        for (int j = 0; j < lt.nt; ++j) v += (T)lt.c[j] * lt.src[j][e];
        const double sc = atol + rtol * fmax(fabs((double)y[e]), fabs((double)y5[e]));
        r = fabs((double)v) / sc;
    }
    for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_max_finish(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double red[4];
    double r = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) r = fmax(r, part[b]);
    for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Size and centre-of-mass constraints of the regularised objective (Eq. 9):
// block sums of psi, psi x and psi y (fixed order), then J and the gradient
// dJ/dpsi_i = c0 + c1 (x_i - x_c) + c2 (y_i - y_c).
template <typename T>
__global__ __launch_bounds__(256) void k_shape_sums(const T* __restrict__ psi, int nx, int ny, int N,
                                                    double* __restrict__ part) {
    __shared__ double red[3][4];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, bx = 0.0, by = 0.0;
    if (i < N) {
        const double v = (double)psi[i];
        a = v;
        bx = v * (double)(i % nx);
        by = v * (double)((i / nx) % ny);
    }
    a = wave_sum(a);
    bx = wave_sum(bx);
    by = wave_sum(by);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = bx;
        red[2][threadIdx.x >> 6] = by;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        part[3 * (size_t)blockIdx.x + k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    }
}

__global__ __launch_bounds__(256) void k_shape_finish(const double* __restrict__ part, int nb, int nz, double xi,
                                                      double S_target, double nu, double x0, double y0,
                                                      double* __restrict__ J, double* __restrict__ coef) {
    __shared__ double red[3][4];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int k = 0; k < 3; ++k) s[k] += part[3 * (size_t)b + k];
    for (int k = 0; k < 3; ++k) {
        const double v = wave_sum(s[k]);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double tot = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    const double sx = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    const double sy = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
    const double S = tot / nz;
    // no material: no centre (the centre constraint and its gradient vanish)
    const double xc = tot > 0.0 ? sx / tot : x0, yc = tot > 0.0 ? sy / tot : y0;
    const double dxc = xc - x0, dyc = yc - y0;
    J[0] = xi * (S - S_target) * (S - S_target) + nu * (fabs(dxc) + fabs(dyc));
    coef[0] = 2.0 * xi * (S - S_target) / nz;
    coef[1] = tot > 0.0 ? nu * (dxc > 0.0 ? 1.0 : (dxc < 0.0 ? -1.0 : 0.0)) / tot : 0.0;
    coef[2] = tot > 0.0 ? nu * (dyc > 0.0 ? 1.0 : (dyc < 0.0 ? -1.0 : 0.0)) / tot : 0.0;
    coef[3] = xc;
    coef[4] = yc;
}

__global__ __launch_bounds__(256) void k_shape_grad(int nx, int ny, int N, const double* __restrict__ coef,
                                                    double* __restrict__ g) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double x = (double)(i % nx), y = (double)((i / nx) % ny);
    g[i] = coef[0] + coef[1] * (x - coef[3]) + coef[2] * (y - coef[4]);
}

// ---------------------------------------------------------------------------
// energy + area objective (single instance): energy terms, dJ/dm and the
// explicit dJ/dpsi, with per-block partial sums (ex, d, Z, an, psi)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) k_energy(const BatchArgs<T> ba, double t, const T* __restrict__ m,
                                                double scale, T* __restrict__ dJdm, double* __restrict__ dJdpsi) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* Z = reinterpret_cast<C*>(smem_raw);
    __shared__ double red[5][512 / 64];
    const int2 wk = ba.single ? make_int2(0, (int)blockIdx.x) : ba.work[blockIdx.x];
    const KParams<T> p = ba.ptab[wk.x];
    const InstTab& tb = ba.itab[wk.x];
    const T* __restrict__ psi = role<T>(tb, B_PSI);
    const uint8_t* antenna = p.has_ant ? role<uint8_t>(tb, B_ANT) : nullptr;
    const int r0 = 2 * wk.y;
    const bool v1 = r0 + 1 < p.nrows;
    const int Px = p.Px;
    constexpr int MR = MaxReg<T>::v;
    const bool demag = (p.terms & 2) != 0;
    if (demag) {
        unpack_rows_to_lds(p, role<C>(tb, B_S), r0, v1, Z);
        __syncthreads();
        fft_lds<C, true, MR>(Z, SigMap{0, ilog2_rt(Px)}, Px, 3, role<C>(tb, B_TWX));
    }
    const T drv = (T)drive_value(p.f1, p.f2, p.t_switch, p.drive_kind, p.t_ramp, t);
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
                const C z01 = Z[lp(x) + lp(rr * Px)];
                const C z2 = Z[lp(x) + lp(2 * Px)];
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
        double* part = role<double>(tb, B_EPART);
        for (int q = 0; q < 5; ++q) {
            double s = 0.0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[q][k];
            part[5 * wk.y + q] = s;
        }
    }
}

// Single-block fixed-order reduction of the energy partials (units of Ms V).
template <typename T>
__global__ void k_energy_finish(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab, double MsV,
                                double lam, double area, double E_ref, double* __restrict__ J,
                                double* __restrict__ en) {
    __shared__ double red[5][256];
    const KParams<T>& p = ptab[0];
    const InstTab& tb = itab[0];
    const double* part = role<double>(tb, B_EPART);
    double s[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < p.nloc; b += blockDim.x)
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
        const double mean = red[4][0] / p.N;
        if (en) {
            en[0] = ex;
            en[1] = d;
            en[2] = z;
            en[3] = an;
            en[4] = ex + d + z + an;
        }
        const double Jv = (ex + d) / E_ref + lam * (mean - area) * (mean - area);
        if (J) *J = Jv;
        double* sc = role<double>(tb, B_SCAL);
        sc[0] = Jv;
        sc[1] = 2.0 * lam * (mean - area) / p.N;
    }
}

template <typename T>
__global__ void k_add_area(const KParams<T>* __restrict__ ptab, const InstTab* __restrict__ itab,
                           double* __restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ptab[0].N) g[i] += role<double>(itab[0], B_SCAL)[1];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
static BatchArgs<T> bargs(const BatchDev<T>& b, const int2* work) {
    BatchArgs<T> a;
    a.ptab = b.ptab;
    a.itab = b.itab;
    a.work = work;
    a.single = b.ninst == 1;
    return a;
}
// Variants by largest FFT radix (4, 8, or 16 in float): the launchers pick
// the one the batch's launch configuration names.
template <typename T, int MR>
static void stage_fwd_r(const BatchDev<T>& b, const FwdL& L, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (L.lin_out) {
        if (b.fwd_rows)
            hipExtLaunchKernelGGL((k_stage_fwd<T, MR, true, true>), dim3(b.nloc), dim3(b.loc_threads), (uint32_t)b.fwd_lds,
                                  s, e0, e1, 0, bargs(b, b.work_loc), L);
        else
            hipExtLaunchKernelGGL((k_stage_fwd<T, MR, false, true>), dim3(b.nloc), dim3(b.loc_threads),
                                  (uint32_t)b.fwd_lds, s, e0, e1, 0, bargs(b, b.work_loc), L);
        return;
    }
    if (b.fwd_rows)
        hipExtLaunchKernelGGL((k_stage_fwd<T, MR, true>), dim3(b.nloc), dim3(b.loc_threads), (uint32_t)b.fwd_lds, s, e0,
                              e1, 0, bargs(b, b.work_loc), L);
    else
        hipExtLaunchKernelGGL((k_stage_fwd<T, MR, false>), dim3(b.nloc), dim3(b.loc_threads), (uint32_t)b.fwd_lds, s,
                              e0, e1, 0, bargs(b, b.work_loc), L);
}
template <typename T, int MR>
static void stage_bwd_r(const BatchDev<T>& b, const BwdL& L, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (L.lin_nt > 0)
        hipExtLaunchKernelGGL((k_stage_bwd<T, MR, true>), dim3(b.nloc), dim3(b.bwd_threads), (uint32_t)b.bwd_lds, s, e0,
                              e1, 0, bargs(b, b.work_loc), L);
    else
        hipExtLaunchKernelGGL((k_stage_bwd<T, MR>), dim3(b.nloc), dim3(b.bwd_threads), (uint32_t)b.bwd_lds, s, e0, e1,
                              0, bargs(b, b.work_loc), L);
}
template <typename T, int NZ, int MR>
static void col_r(const BatchDev<T>& b, int spec, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (NZ == 1)
        hipExtLaunchKernelGGL((k_col2d<T, MR>), dim3(b.ncol), dim3(b.col_threads), (uint32_t)b.col_lds, s, e0, e1, 0,
                              bargs(b, b.work_col), b.col_tk, spec, b.col_nt_lds);
    else
        hipExtLaunchKernelGGL((k_col_conv<T, NZ, MR>), dim3(b.ncol), dim3(b.col_threads), (uint32_t)b.col_lds, s, e0,
                              e1, 0, bargs(b, b.work_col), b.col_tk, spec, b.col_nt_lds);
}
template <typename T, int NZ>
static void col_nz(const BatchDev<T>& b, int spec, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (b.col_radix == 4)
        col_r<T, NZ, 4>(b, spec, s, e0, e1);
    else if (b.col_radix == 8 || sizeof(T) == 8)
        col_r<T, NZ, 8>(b, spec, s, e0, e1);
    else
        col_r<T, NZ, MaxReg<T>::v>(b, spec, s, e0, e1);
}

template <typename T>
hipError_t launch_stage_fwd(const BatchDev<T>& b, const FwdL& L, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (b.loc_radix == 4)
        stage_fwd_r<T, 4>(b, L, s, e0, e1);
    else if (b.loc_radix == 8 || sizeof(T) == 8)
        stage_fwd_r<T, 8>(b, L, s, e0, e1);
    else
        stage_fwd_r<T, MaxReg<T>::v>(b, L, s, e0, e1);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_stage_bwd(const BatchDev<T>& b, const BwdL& L, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    BwdL Lm = L;
    Lm.stage_m = b.loc_nv >= 7;
    if (b.bwd_radix == 4)
        stage_bwd_r<T, 4>(b, Lm, s, e0, e1);
    else if (b.bwd_radix == 8 || sizeof(T) == 8)
        stage_bwd_r<T, 8>(b, Lm, s, e0, e1);
    else
        stage_bwd_r<T, MaxReg<T>::v>(b, Lm, s, e0, e1);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_col_conv(const BatchDev<T>& b, int max_nz, int spec, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (max_nz == 1)
        col_nz<T, 1>(b, spec, s, e0, e1);
    else if (max_nz == 2)
        col_nz<T, 2>(b, spec, s, e0, e1);
    else if (max_nz <= 4)
        col_nz<T, 4>(b, spec, s, e0, e1);
    else
        col_nz<T, 8>(b, spec, s, e0, e1);
    return hipGetLastError();
}
// Registers per lane of the column-kernel variant a launch with these
// parameters would run (0 if the runtime cannot say).
template <typename T>
int col_conv_vgprs(int max_nz, int radix) {
    const void* f;
    constexpr int RT = MaxReg<T>::v;
    const int r = radix == 4 ? 4 : (radix == 8 || sizeof(T) == 8) ? 8 : RT;
    const int z = max_nz == 1 ? 1 : max_nz == 2 ? 2 : max_nz <= 4 ? 4 : 8;
#define LLG_PICK(Z)                                                                                   \
    if (z == Z)                                                                                       \
        f = r == 4 ? reinterpret_cast<const void*>(k_col_conv<T, Z, 4>)                               \
                   : r == 8 ? reinterpret_cast<const void*>(k_col_conv<T, Z, 8>)                      \
                            : reinterpret_cast<const void*>(k_col_conv<T, Z, RT>);
    if (z == 1)
        f = r == 4 ? reinterpret_cast<const void*>(k_col2d<T, 4>)
                   : r == 8 ? reinterpret_cast<const void*>(k_col2d<T, 8>) : reinterpret_cast<const void*>(k_col2d<T, RT>);
    else LLG_PICK(2) else LLG_PICK(4) else LLG_PICK(8)
#undef LLG_PICK
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, f) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return at.numRegs;
}

template <typename T>
int stage_fwd_vgprs(int radix, int staged) {
    constexpr int RT = MaxReg<T>::v;
    const int r = radix == 4 ? 4 : (radix == 8 || sizeof(T) == 8) ? 8 : RT;
    const void* f;
    if (staged)
        f = r == 4 ? reinterpret_cast<const void*>(k_stage_fwd<T, 4, true>)
            : r == 8 ? reinterpret_cast<const void*>(k_stage_fwd<T, 8, true>)
                     : reinterpret_cast<const void*>(k_stage_fwd<T, RT, true>);
    else
        f = r == 4 ? reinterpret_cast<const void*>(k_stage_fwd<T, 4, false>)
            : r == 8 ? reinterpret_cast<const void*>(k_stage_fwd<T, 8, false>)
                     : reinterpret_cast<const void*>(k_stage_fwd<T, RT, false>);
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, f) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return at.numRegs;
}

template <typename T>
static dim3 elem_grid(const BatchDev<T>& b, int per_inst) {
    return dim3((unsigned)((per_inst + 255) / 256), (unsigned)b.ninst);
}
template <typename T>
hipError_t launch_levelset(const BatchDev<T>& b, double a, int extrude, hipStream_t s) {
    hipLaunchKernelGGL(k_levelset<T>, elem_grid(b, b.max_n3 / 3), dim3(256), 0, s, b.ptab, b.itab, (T)a, extrude);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_levelset_vjp(const BatchDev<T>& b, double a, int extrude, hipStream_t s) {
    hipLaunchKernelGGL(k_levelset_vjp<T>, elem_grid(b, b.max_n3 / 3), dim3(256), 0, s, b.ptab, b.itab, a, extrude);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_init(const BatchDev<T>& b, int lam_sel, int use_djdm, int port, int W, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_init<T>, elem_grid(b, b.max_n3 / 3), dim3(256), 0, s, b.ptab, b.itab, lam_sel, use_djdm,
                       port, W);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_psi_grad_out(const BatchDev<T>& b, int use_expl, hipStream_t s) {
    hipLaunchKernelGGL(k_psi_grad_out<T>, elem_grid(b, b.max_n3 / 3), dim3(256), 0, s, b.ptab, b.itab, use_expl);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_zero(const BatchDev<T>& b, int sel, int what, hipStream_t s) {
    const int n = what == 0 ? b.max_n3 / 3 : 2 * b.nloc;
    hipLaunchKernelGGL(k_zero<T>, elem_grid(b, n), dim3(256), 0, s, b.ptab, b.itab, sel, what);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_fill(const BatchDev<T>& b, int sel, int mult, double v, hipStream_t s, int off) {
    hipLaunchKernelGGL(k_fill<T>, elem_grid(b, mult * (b.max_n3 / 3)), dim3(256), 0, s, b.ptab, b.itab, sel, mult, (T)v,
                       off);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_copy(const BatchDev<T>& b, int src, int src_slot, int dst, int dst_slot, int mult, hipStream_t s) {
    hipLaunchKernelGGL(k_copy<T>, elem_grid(b, mult * b.max_n3), dim3(256), 0, s, b.ptab, b.itab, src, src_slot, dst,
                       dst_slot, mult);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_port_finish(const BatchDev<T>& b, int W, hipStream_t s) {
    hipLaunchKernelGGL(k_port_finish<T>, dim3(b.ninst), dim3(256), 0, s, b.ptab, b.itab, W);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_lincomb(int n, T* out, const T* base, const LinTerms<T>& lt, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, out, base, lt);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_err_norm(int n, const T* y, const T* y5, const LinTerms<T>& lt, double rtol, double atol,
                           double* part, double* out, hipStream_t s) {
    const int nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_err_norm<T>, dim3(nb), dim3(256), 0, s, n, y, y5, lt, rtol, atol, part);
    hipLaunchKernelGGL(k_max_finish, dim3(1), dim3(256), 0, s, part, nb, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_shape(const T* psi, int nx, int ny, int nz, double xi, double S_target, double nu, double x0,
                        double y0, double* work, double* J, double* g, hipStream_t s) {
    const int N = nx * ny * nz, nb = (N + 255) / 256;
    hipLaunchKernelGGL(k_shape_sums<T>, dim3(nb), dim3(256), 0, s, psi, nx, ny, N, work + 8);
    hipLaunchKernelGGL(k_shape_finish, dim3(1), dim3(256), 0, s, work + 8, nb, nz, xi, S_target, nu, x0, y0, J, work);
    if (g) hipLaunchKernelGGL(k_shape_grad, dim3(nb), dim3(256), 0, s, nx, ny, N, work, g);
    return hipGetLastError();
}
// File-scope scratch of the allocation-free shape-penalty call: the block
// partial sums (3 per 256 nodes) and the five finishing coefficients of at most
// kShapeMaxNodes nodes.  One copy per GPU, held until the process ends.  Host
// code never passes `scratch` itself to a kernel (in host code the name is a
// host-side stand-in); it passes the per-device address that
// hipGetSymbolAddress returns.
constexpr int kShapeScratchDoubles = 8 + 3 * ((kShapeMaxNodes + 255) / 256);
static __device__ __align__(256) double scratch[kShapeScratchDoubles];

hipError_t shape_scratch_ptr(double** out) {
    static std::mutex mu;
    static double* ptrs[64] = {nullptr};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptrs[dev] = static_cast<double*>(p);
    }
    *out = ptrs[dev];
    return hipSuccess;
}

template <typename T>
hipError_t launch_curve(const BatchDev<T>& b, const double* tw, int W, hipStream_t s) {
    hipLaunchKernelGGL(k_curve_series<T>, dim3((W + 255) / 256, b.ninst), dim3(256), 0, s, b.ptab, b.itab, tw, W);
    hipLaunchKernelGGL(k_curve_finish<T>, dim3(b.ninst), dim3(256), 0, s, b.ptab, b.itab, tw, W);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_spectral(const BatchDev<T>& b, const double* fc, int K, int W, double t0, int64_t n_start, double dt,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_spec_series<T>, dim3(W, b.ninst), dim3(64), 0, s, b.ptab, b.itab);
    hipLaunchKernelGGL(k_spec_dft<T>, dim3(K, b.ninst), dim3(256), 0, s, b.ptab, b.itab, fc, W, t0, n_start, dt);
    hipLaunchKernelGGL(k_spec_finish<T>, dim3(b.ninst), dim3(64), 0, s, b.ptab, b.itab, fc, K);
    hipLaunchKernelGGL(k_spec_src<T>, dim3((W + 255) / 256, b.ninst), dim3(256), 0, s, b.ptab, b.itab, fc, K, W, t0,
                       n_start, dt);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_energy(const BatchDev<T>& b, double t, const T* m, double scale, T* dJdm, double* dJdpsi,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_energy<T>, dim3(b.nloc), dim3(b.loc_threads), b.loc_lds, s, bargs(b, b.work_loc), t, m,
                       scale, dJdm, dJdpsi);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_energy_finish(const BatchDev<T>& b, double MsV, double lam, double area, double E_ref, double* J,
                                double* en, double* dJdpsi, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_finish<T>, dim3(1), dim3(256), 0, s, b.ptab, b.itab, MsV, lam, area, E_ref, J, en);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !dJdpsi) return e;
    hipLaunchKernelGGL(k_add_area<T>, elem_grid(b, b.max_n3 / 3), dim3(256), 0, s, b.ptab, b.itab, dJdpsi);
    return hipGetLastError();
}

// The dynamic-LDS limit is a per-kernel attribute shared by every handle of
// the process: it only ever grows, so a handle never lowers another's limit.
template <typename T>
hipError_t set_lds_limits(size_t bytes) {
    static std::mutex mu;
    static size_t current = 65536;
    std::lock_guard<std::mutex> lock(mu);
    if (bytes <= current) return hipSuccess;
    hipError_t e = hipSuccess;
    const int v = (int)bytes;
#define LLG_ATTR(K) \
    if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void*>(K), hipFuncAttributeMaxDynamicSharedMemorySize, v);
    constexpr int RT = MaxReg<T>::v;
    LLG_ATTR((k_stage_fwd<T, 4, true>))
    LLG_ATTR((k_stage_fwd<T, 8, true>))
    LLG_ATTR((k_stage_fwd<T, RT, true>))
    LLG_ATTR((k_stage_fwd<T, 4, false>))
    LLG_ATTR((k_stage_fwd<T, 8, false>))
    LLG_ATTR((k_stage_fwd<T, RT, false>))
    LLG_ATTR((k_stage_fwd<T, 4, true, true>))
    LLG_ATTR((k_stage_fwd<T, 8, true, true>))
    LLG_ATTR((k_stage_fwd<T, RT, true, true>))
    LLG_ATTR((k_stage_fwd<T, 4, false, true>))
    LLG_ATTR((k_stage_fwd<T, 8, false, true>))
    LLG_ATTR((k_stage_fwd<T, RT, false, true>))
    LLG_ATTR((k_stage_bwd<T, 4>))
    LLG_ATTR((k_stage_bwd<T, 8>))
    LLG_ATTR((k_stage_bwd<T, RT>))
    LLG_ATTR((k_stage_bwd<T, 4, true>))
    LLG_ATTR((k_stage_bwd<T, 8, true>))
    LLG_ATTR((k_stage_bwd<T, RT, true>))
    LLG_ATTR((k_col2d<T, 4>))
    LLG_ATTR((k_col2d<T, 8>))
    LLG_ATTR((k_col2d<T, RT>))
    LLG_ATTR((k_col_conv<T, 2, 4>))
    LLG_ATTR((k_col_conv<T, 4, 4>))
    LLG_ATTR((k_col_conv<T, 8, 4>))
    LLG_ATTR((k_col_conv<T, 2, 8>))
    LLG_ATTR((k_col_conv<T, 4, 8>))
    LLG_ATTR((k_col_conv<T, 8, 8>))
    LLG_ATTR((k_col_conv<T, 2, RT>))
    LLG_ATTR((k_col_conv<T, 4, RT>))
    LLG_ATTR((k_col_conv<T, 8, RT>))
    LLG_ATTR(k_energy<T>)
#undef LLG_ATTR
    if (e == hipSuccess) current = bytes;
    return e;
}

#define LLG_INST(T)                                                                                                 \
    template hipError_t launch_stage_fwd<T>(const BatchDev<T>&, const FwdL&, hipStream_t, hipEvent_t, hipEvent_t);  \
    template hipError_t launch_stage_bwd<T>(const BatchDev<T>&, const BwdL&, hipStream_t, hipEvent_t, hipEvent_t);  \
    template hipError_t launch_col_conv<T>(const BatchDev<T>&, int, int, hipStream_t, hipEvent_t, hipEvent_t);      \
    template int col_conv_vgprs<T>(int, int);                                                                       \
    template int stage_fwd_vgprs<T>(int, int);                                                                           \
    template hipError_t launch_levelset<T>(const BatchDev<T>&, double, int, hipStream_t);                           \
    template hipError_t launch_levelset_vjp<T>(const BatchDev<T>&, double, int, hipStream_t);                       \
    template hipError_t launch_adj_init<T>(const BatchDev<T>&, int, int, int, int, hipStream_t);                     \
    template hipError_t launch_psi_grad_out<T>(const BatchDev<T>&, int, hipStream_t);                               \
    template hipError_t launch_zero<T>(const BatchDev<T>&, int, int, hipStream_t);                                  \
    template hipError_t launch_fill<T>(const BatchDev<T>&, int, int, double, hipStream_t, int);                         \
    template hipError_t launch_copy<T>(const BatchDev<T>&, int, int, int, int, int, hipStream_t);                        \
    template hipError_t launch_port_finish<T>(const BatchDev<T>&, int, hipStream_t);                                \
    template hipError_t launch_curve<T>(const BatchDev<T>&, const double*, int, hipStream_t);                      \
    template hipError_t launch_lincomb<T>(int, T*, const T*, const LinTerms<T>&, hipStream_t);                    \
    template hipError_t launch_err_norm<T>(int, const T*, const T*, const LinTerms<T>&, double, double, double*,   \
                                           double*, hipStream_t);                                                   \
    template hipError_t launch_shape<T>(const T*, int, int, int, double, double, double, double, double, double*,  \
                                        double*, double*, hipStream_t);                                             \
    template hipError_t launch_spectral<T>(const BatchDev<T>&, const double*, int, int, double, int64_t, double,     \
                                           hipStream_t);                                                            \
    template hipError_t launch_energy<T>(const BatchDev<T>&, double, const T*, double, T*, double*, hipStream_t);   \
    template hipError_t launch_energy_finish<T>(const BatchDev<T>&, double, double, double, double, double*,        \
                                                double*, double*, hipStream_t);                                     \
    template hipError_t set_lds_limits<T>(size_t);

LLG_INST(float)
LLG_INST(double)

}  // namespace llg
