// Host runtime of the level-set LLG library: batches of problem instances,
// their device workspace and tables, argument validation, stream-ordered
// orchestration of the forward run, the objectives and the checkpointed
// discrete adjoint, and the extern "C" entry points.  A single-instance
// handle is a batch of one; every launch serves all instances of a batch.
//
// Discrete adjoint (the exact gradient of the fixed-step RK4 map; the discrete
// counterpart of the paper's adjoint system, Eq. 6, and gradient integral,
// Eq. 7).  With lambda' = dJ/dm_{n+1} and the stage states y_1..y_4 of step n:
//   l_4 = dt/6 lambda',  l_3 = dt/3 lambda' + dt mu_4,  l_2 = dt/3 lambda' + dt/2 mu_3,
//   l_1 = dt/6 lambda' + dt/2 mu_2,  mu_s = J_f(y_s)^T l_s,
//   lambda_n = lambda' + sum_s mu_s (+ running-cost source),  dJ/dpsi += sum_s l_s . df/dpsi(y_s).
// Each mu_s needs the demag convolution of the field adjoint u_s, so every
// backward stage is one column kernel plus one local kernel, like the forward.
//
// Checkpointing: the forward stores m every K steps.  The adjoint walks the
// segments backwards; for each it restores the snapshot, re-runs the K steps
// while storing every stage state and field (bitwise identical to the first
// run: same kernels, same launch shapes, no atomics), then runs the K backward
// steps.  Memory: ceil(n/K) snapshots + 8K stage vectors; K ~ sqrt(n).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/llg.h"
#include "llg_internal.hpp"
#include "llg_schedule.hpp"

using namespace llg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(LLG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

int pow2_at_least(long long v) {
    int p = 1;
    while (p < v) p *= 2;
    return p;
}
int padded(int n) { return n == 1 ? 1 : pow2_at_least(2LL * n - 1); }
int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Instance {
    llg_problem prob{};
    int N = 0, nrows = 0, Px = 1, Py = 1, Pz = 1, Kx = 1, ncomp = 4;
    int ktiles = 1;  // x-bin tiles of the stored spectra
    int pack = 0;    // bins 0 and Px/2 transformed as one column (see column_work)
    int nloc = 0;
    long long n_p1 = 0, n_p2 = 0;
    bool has_ant = false, has_design = false;
    KParams<float> pf{};
    KParams<double> pd{};
    InstTab tab{};
};

}  // namespace

struct llg_handle {
    int dtype = LLG_F32;
    size_t tsz = 4;
    bool demag = false;
    int terms = 0;
    std::vector<Instance> inst;
    std::vector<DevBuf> bufs;
    // device tables
    void* ptab = nullptr;
    InstTab* itab = nullptr;
    int2* work_loc = nullptr;
    int2* work_col = nullptr;
    BatchDev<float> bf{};
    BatchDev<double> bd{};
    int max_nz = 1;
    // byte sums over instances (profiling)
    double sumN = 0, sumSpec = 0, sumNhat = 0;
    // checkpoint store: nsnap snapshot slots, K stage-state slots per half, halves = 2
    // when consecutive segments are recomputed and transposed concurrently
    int64_t K = 1, nsnap = 0, halves = 1;
    int32_t policy = LLG_CKPT_SQRT, ckpt_param = 0;
    int64_t max_steps = 1;
    Plan plan;  // binomial schedule of the last forward run
    int64_t plan_n = -1;
    int plan_slots = 0;
    // second stream (segment recomputation) and its synchronisation events
    hipStream_t aux = nullptr;
    std::vector<hipEvent_t> sync_ev;
    // HIP graphs of the forward / adjoint launch sequences, keyed by the call
    // signature; captured and replayed on a stream of the handle
    struct GraphEntry {
        std::vector<double> key;
        hipGraphExec_t exec;
        int result;
    };
    bool graphs_on = false;
    hipStream_t gstream = nullptr;
    hipEvent_t g_in = nullptr, g_out = nullptr;
    std::vector<GraphEntry> graphs;
    // per-kernel profiling
    struct ProfRec { int kind; double bytes; hipEvent_t a, b; };
    bool prof_on = false;
    int prof_stride = 1;                      // bracket every prof_stride-th launch of each class
    int64_t prof_seen[LLG_KIND_COUNT] = {0};  // launches of each class since profiling was enabled
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[LLG_KIND_COUNT] = {0};
    double prof_bytes[LLG_KIND_COUNT] = {0};
    int64_t prof_n[LLG_KIND_COUNT] = {0};
    // spectral objective: sample frequencies and weights on the device (f, c_1, c_2)
    double* spec_fc = nullptr;
    int spec_cap = 0;        // capacity in frequencies of spec_fc and of every instance's B_SPC
    int spec_k = 0;          // frequencies of the last upload
    std::vector<double> spec_host;
    // curve objective: targets and weights of the window steps on the device
    double* curve_tw = nullptr;
    double* shape_work = nullptr;  // size / centre constraints: coefficients and block sums
    // adaptive Dormand-Prince run: stage rates, trial state, per-step snapshots,
    // stage adjoints, error-norm scratch; the accepted steps of the last run
    struct Dopri {
        void* k[7] = {};
        void* y5 = nullptr;
        void* ystage = nullptr;
        void* ystage2 = nullptr;  // stage states alternate between the two while one is read
        void* snaps = nullptr;   // (max_steps + 1) states
        void* mu[6] = {};
        void* lam = nullptr;
        double* err = nullptr;   // [0] norm, [8..] block maxima
        double* err_host = nullptr;  // pinned host copy of the norm, read after each trial step
        std::vector<double> hs, ts;
        bool valid = false;
        // optional store of every accepted step's stages, 11 state vectors per step n:
        // B_0, then (Y_s, B_s) for s = 1..5 (Y_0 is the kept state); max_steps + 1 steps
        void* stages = nullptr;
        bool keep = false;         // the next adaptive run fills the store
        bool stages_valid = false;  // the last adaptive run filled it
    } dp;
    std::vector<double> curve_host;
    // forward record
    bool fwd_valid = false;
    double t0 = 0.0;
    int64_t n_steps = 0;
    int64_t K_used = 1;
    llg_objective_spec last_obj{};
};

namespace {

template <typename T> KParams<T>& kp(Instance& I);
template <> KParams<float>& kp<float>(Instance& I) { return I.pf; }
template <> KParams<double>& kp<double>(Instance& I) { return I.pd; }
template <typename T> BatchDev<T>& bdev(llg_handle* h);
template <> BatchDev<float>& bdev<float>(llg_handle* h) { return h->bf; }
template <> BatchDev<double>& bdev<double>(llg_handle* h) { return h->bd; }

int alloc(llg_handle* h, void** out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) return LLG_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LLG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    h->bufs.push_back({p, bytes});
    *out = p;
    return LLG_OK;
}

void free_all(llg_handle* h) {
    for (auto& b : h->bufs) (void)hipFree(b.p);
    h->bufs.clear();
}

template <typename T>
void fill_params(Instance& I) {
    KParams<T>& p = kp<T>(I);
    const llg_problem& q = I.prob;
    p.nx = q.nx;
    p.ny = q.ny;
    p.nz = q.nz;
    p.N = I.N;
    p.nrows = I.nrows;
    p.Px = I.Px;
    p.Kx = I.Kx;
    p.Py = I.Py;
    p.Pz = I.Pz;
    p.Ky2 = I.Py / 2 + 1;
    p.Kz2 = I.Pz / 2 + 1;
    p.ktiles = I.ktiles;
    p.pack = I.pack;
    p.ncomp = I.ncomp;
    p.terms = q.terms;
    p.nloc = I.nloc;
    p.has_ant = I.has_ant;
    p.n_p1 = (int)I.n_p1;
    p.n_p2 = (int)I.n_p2;
    const double kappa = 2.0 * q.A / q.Ms;
    const double hh[3] = {q.dx, q.dy, q.dz};
    for (int d = 0; d < 3; ++d) p.exw[d] = (T)(2.0 * kappa / (hh[d] * hh[d]));
    p.anis = (T)(2.0 * q.K / q.Ms);
    const double un = std::sqrt(q.ku[0] * q.ku[0] + q.ku[1] * q.ku[1] + q.ku[2] * q.ku[2]);
    for (int d = 0; d < 3; ++d) {
        p.u[d] = (T)(un > 0 ? q.ku[d] / un : 0.0);
        p.B0[d] = (T)q.B0[d];
        p.brf[d] = (T)q.b_rf[d];
    }
    p.alpha0 = (T)q.alpha0;
    p.alpha_max = (T)q.alpha_max;
    p.ramp_cells = q.ramp_cells;
    p.ramp_faces = q.ramp_faces;
    p.gamma = (T)q.gamma;
    p.dt = (T)q.dt;
    p.f1 = q.f1;
    p.f2 = q.f2;
    p.t_switch = q.t_switch;
    p.drive_kind = q.drive_kind;
    p.t_ramp = q.t_ramp;
    p.psi_freeze = (T)q.psi_freeze;
}

template <typename T>
int upload_tables(llg_handle* h, Instance& I) {
    using C = cplx<T>;
    auto twiddles = [&](int L, int id) -> int {
        std::vector<C> tw(L);
        for (int k = 0; k < L; ++k) {
            const double th = -2.0 * 3.14159265358979323846 * (double)k / (double)L;
            tw[k].x = (T)std::cos(th);
            tw[k].y = (T)std::sin(th);
        }
        int rc = alloc(h, &I.tab.b[id], sizeof(C) * L);
        if (rc) return rc;
        HIPCHK(hipMemcpy(I.tab.b[id], tw.data(), sizeof(C) * L, hipMemcpyHostToDevice));
        return LLG_OK;
    };
    int rc;
    if ((rc = twiddles(I.Px, B_TWX))) return rc;
    if ((rc = twiddles(I.Py, B_TWY))) return rc;
    if ((rc = twiddles(I.Pz, B_TWZ))) return rc;
    if (h->demag) {
        const llg_problem& q = I.prob;
        const double scale = -kMu0 * q.Ms / ((double)I.Px * I.Py * I.Pz);
        // instances with the same grid, cells and Ms (e.g. one design at several
        // frequencies) share one device copy of the tensor spectrum
        const std::vector<double> key = {(double)q.nx, (double)q.ny, (double)q.nz, q.dx, q.dy, q.dz, scale};
        for (const Instance& J : h->inst) {
            if (&J == &I || !J.tab.b[B_NHAT]) continue;
            const llg_problem& r = J.prob;
            const double sj = -kMu0 * r.Ms / ((double)J.Px * J.Py * J.Pz);
            const std::vector<double> kj = {(double)r.nx, (double)r.ny, (double)r.nz, r.dx, r.dy, r.dz, sj};
            if (kj == key) {
                I.tab.b[B_NHAT] = J.tab.b[B_NHAT];
                I.ncomp = J.ncomp;
                return LLG_OK;
            }
        }
        std::vector<double> spec;
        int nc = 4;
        build_tensor_spectrum(q.nx, q.ny, q.nz, q.dx, q.dy, q.dz, I.Px, I.Py, I.Pz, scale, spec, nc);
        I.ncomp = nc;
        // into 128-byte x-bin tiles: [(t * NR + q) * TW + o], q = (comp * Kz2 + kz) * Ky2 + ky
        const int TW = spec_tile<T>();
        const size_t NR = spec.size() / I.Kx;
        std::vector<T> st((size_t)I.ktiles * NR * TW, (T)0);
        for (size_t q = 0; q < NR; ++q)
            for (int kx = 0; kx < I.Kx; ++kx)
                st[((size_t)(kx / TW) * NR + q) * TW + kx % TW] = (T)spec[q * I.Kx + kx];
        if ((rc = alloc(h, &I.tab.b[B_NHAT], sizeof(T) * st.size()))) return rc;
        HIPCHK(hipMemcpy(I.tab.b[B_NHAT], st.data(), sizeof(T) * st.size(), hipMemcpyHostToDevice));
    }
    return LLG_OK;
}

// ---------------------------------------------------------------------------
// launch geometry: one configuration for the whole batch (the most demanding
// instance sets the minimum block sizes and the LDS); every valid
// configuration computes identical bits (same FFT passes per signal, same
// per-node arithmetic), only the tiling of the work over blocks changes
// ---------------------------------------------------------------------------
struct LaunchCfg {
    int tk = 1;        // column-kernel tile: x-bins per block
    int col_thr = 64;
    int col_r = 16;    // largest FFT radix of the column kernel (4, 8, 16; 16 in float only)
    int fwd_thr = 64;  // forward row kernel
    int fwd_r = 16;
    int bwd_thr = 64;  // backward row kernel
    int bwd_r = 16;
    int nv = 4;        // node values per staged row in the backward row kernel (4: u, psi; 7: also y_s)
};

int maxreg_of(const llg_handle* h) { return h->dtype == LLG_F32 ? 16 : 8; }
bool radix_ok(const llg_handle* h, int r) { return r == 4 || r == 8 || (r == 16 && h->dtype == LLG_F32); }

// fewest threads the row kernels need (FFT register budget of radix r), at least 64
int loc_min_threads(const llg_handle* h, int r) {
    int thr = 64;
    for (auto& I : h->inst) thr = std::max(thr, round_up((3 * I.Px + r - 1) / r, 64));
    return thr;
}

// LDS of the row kernels with nv node values per staged row (4 rows)
size_t loc_lds_bytes(const llg_handle* h, int nv) {
    size_t lds = 0;
    for (auto& I : h->inst)
        lds = std::max(lds, (h->demag ? (size_t)(lds_pad(3 * I.Px) + I.Px) * 2 * h->tsz : 0) +
                                (size_t)4 * nv * I.prob.nx * h->tsz);
    return lds;
}


// column-kernel LDS: padded columns, twiddles, and (nt = true) the tensor-spectrum tile
size_t col_lds_bytes(const llg_handle* h, const Instance& I, int tk, bool nt) {
    const size_t csz = 2 * h->tsz;
    const int Ky2 = I.Py / 2 + 1, Kz2 = I.Pz / 2 + 1;
    return (size_t)lds_pad(3 * I.prob.nz * I.Py * tk) * csz + (size_t)I.Py * csz +
           (nt ? (size_t)I.ncomp * Kz2 * Ky2 * tk * h->tsz : 0);
}

// the tile is staged when every instance's column block then still fits
bool col_nt_lds(const llg_handle* h, int tk) {
    for (auto& I : h->inst)
        if (col_lds_bytes(h, I, tk, true) > 163840) return false;
    return true;
}

size_t col_lds_bytes(const llg_handle* h, const Instance& I, int tk) {
    return col_lds_bytes(h, I, tk, col_nt_lds(h, tk));
}

int col_min_threads(const llg_handle* h, int tk, int r) {
    int thr = 64;
    for (auto& I : h->inst) thr = std::max(thr, round_up((3 * I.prob.nz * I.Py * tk + r - 1) / r, 64));
    return thr;
}

// block-size limit of the column kernel variant with largest radix r (its
// launch bound): radix 16 keeps its butterflies in registers at 512 threads;
// below, up to 4 planes in z fit the registers of 768 threads without spills,
// and 5 to 8 planes need up to 1024 threads for 512-point columns
int col_max_threads(const llg_handle* h, int r) { return r >= 16 ? 512 : h->max_nz > 4 ? 1024 : 768; }

bool col_fits(const llg_handle* h, int tk, int r) {
    for (auto& I : h->inst)
        if (col_lds_bytes(h, I, tk) > 163840) return false;
    return col_min_threads(h, tk, r) <= col_max_threads(h, r);
}

int check_cfg(const llg_handle* h, const LaunchCfg& c) {
    if (!radix_ok(h, c.col_r) || !radix_ok(h, c.fwd_r) || !radix_ok(h, c.bwd_r))
        return fail(LLG_EINVAL, "FFT radix must be 4, 8 or (float only) 16");
    if (c.tk != 1 && c.tk != 2 && c.tk != 4 && c.tk != 8 && c.tk != 16)
        return fail(LLG_EINVAL, "column tile must be 1, 2, 4, 8 or 16");
    if (c.tk > spec_tile_of((int)h->tsz)) return fail(LLG_EINVAL, "column tile wider than a spectrum tile (8 in double)");
    if (!col_fits(h, c.tk, c.col_r)) return fail(LLG_ESHAPE, "column tile " + std::to_string(c.tk) + " does not fit");
    const int cmin = col_min_threads(h, c.tk, c.col_r);
    const int cmax = col_max_threads(h, c.col_r);
    if (c.col_thr % 64 || c.col_thr < cmin || c.col_thr > cmax)
        return fail(LLG_EINVAL, "column threads must be a multiple of 64 in [" + std::to_string(cmin) + ", " +
                                    std::to_string(cmax) + "]");
    for (auto tr : {std::make_pair(c.fwd_thr, c.fwd_r), std::make_pair(c.bwd_thr, c.bwd_r)}) {
        const int lmin = loc_min_threads(h, tr.second);
        if (tr.first % 64 || tr.first < lmin || tr.first > 512)
            return fail(LLG_EINVAL, "row threads must be a multiple of 64 in [" + std::to_string(lmin) + ", 512]");
    }
    if (c.nv != 4 && c.nv != 7) return fail(LLG_EINVAL, "staged row values must be 4 or 7");
    if (loc_lds_bytes(h, c.nv) > 163840) return fail(LLG_ESHAPE, "staged rows do not fit 160 KiB of LDS");
    return LLG_OK;
}

// The rule used at creation: row blocks as wide as the widest row (<= 512),
// column tiles as wide as keeps >= 256 blocks.
int default_cfg(const llg_handle* h, LaunchCfg& c) {
    const int r = maxreg_of(h);
    // column radix: the largest whose block fits the tallest column
    int cr = r;
    while (cr > 4 && !col_fits(h, 1, cr)) cr /= 2;
    int lt = loc_min_threads(h, r);
    for (auto& I : h->inst) lt = std::max(lt, round_up(std::min(I.prob.nx, 512), 64));
    if (loc_min_threads(h, r) > 512)
        return fail(LLG_ESHAPE, "x extent too large for the row kernels");
    if (loc_lds_bytes(h, 4) > 163840) return fail(LLG_ESHAPE, "row kernels need more than 160 KiB of LDS");
    auto blocks_of = [&](int tk) {
        long long b = 0;
        for (auto& I : h->inst) b += (I.Kx - I.pack + tk - 1) / tk;
        return b;
    };
    int tk = std::min(8, spec_tile_of((int)h->tsz));
    while (tk > 1 && (blocks_of(tk) < 256 || !col_fits(h, tk, cr))) tk /= 2;
    if (!col_fits(h, tk, cr)) return fail(LLG_ESHAPE, "y/z extent too large for the column FFT");
    int ct = col_min_threads(h, tk, cr);
    for (auto& I : h->inst)
        ct = std::max(ct, std::min(col_max_threads(h, cr), round_up(std::min(I.Py * tk, 256), 64)));
    c.tk = tk;
    c.col_thr = ct;
    c.col_r = cr;
    c.fwd_thr = c.bwd_thr = lt;
    c.fwd_r = c.bwd_r = r;
    c.nv = 4;
    return LLG_OK;
}

// Make c the batch's launch configuration: column work list, block sizes, LDS limits.
// Column work list: one item per (instance, tile of tk bins).  The tk-bin tiles
// of one 128-byte spectrum tile read the same cache lines, so they are placed
// 8 items apart: thread blocks are dealt round-robin to the 8 XCDs, and this
// keeps a spectrum tile's blocks on one XCD (one L2) and close in time.
// Where an instance packs its real bins (bin Px/2 alone in the last spectrum
// tile, Kx > TW), the block of bin 0 transforms bin Px/2 together with bin 0,
// and that tile gets no item.  Each instance's tiles start at a rotated position so
// that the blocks of bin 0 (which carry the second column) spread over the XCDs.
std::vector<int2> column_work(const llg_handle* h, int tk) {
    const int TW = spec_tile_of((int)h->tsz);
    const int nsub = TW / tk;
    std::vector<int2> tiles;  // (instance, spectrum tile)
    for (int i = 0; i < (int)h->inst.size(); ++i) {
        const int nt = h->inst[i].pack ? h->inst[i].ktiles - 1 : h->inst[i].ktiles;
        for (int t = 0; t < nt; ++t) tiles.push_back(make_int2(i, (t + i) % nt));
    }
    // items past an instance's last bin stay in place as empty blocks (k0 = kNoBin)
    // so that every group keeps the stride of 8
    constexpr int kNoBin = 1 << 30;
    std::vector<int2> wc;
    for (size_t g = 0; g < tiles.size(); g += 8) {
        const size_t ng = std::min<size_t>(8, tiles.size() - g);
        const size_t stride = nsub > 1 ? 8 : ng;
        for (int sub = 0; sub < nsub; ++sub)
            for (size_t j = 0; j < stride; ++j) {
                const int2 tt = tiles[g + std::min(j, ng - 1)];
                const int k0 = tt.y * TW + sub * tk;
                wc.push_back(make_int2(tt.x, j < ng && k0 < h->inst[tt.x].Kx ? k0 : kNoBin));
            }
    }
    return wc;
}

// Blocks of `threads` threads that fit one CU at `lds` bytes of LDS and `regs`
// registers per lane: the lesser of the LDS bound (160 KiB) and the register
// bound (512 registers per SIMD lane, 4 SIMDs, at most 8 waves per SIMD).
int resident_blocks(size_t lds, int regs, int threads) {
    const int waves_simd = regs > 0 ? std::min(8, 512 / round_up(regs, 8)) : 8;
    const int by_regs = std::max(1, 4 * waves_simd / std::max(1, threads / 64));
    const int by_lds = (int)(163840 / std::max<size_t>(lds, 1));
    return std::min(by_lds, by_regs);
}

// The tensor-spectrum tile is staged in LDS only where that costs no resident
// column block per CU; without the tile the kernel reads the tensor from
// memory in the multiply.
bool col_stage_tile(const llg_handle* h, const LaunchCfg& c) {
    if (!col_nt_lds(h, c.tk)) return false;
    size_t with = 0, without = 0;
    for (auto& I : h->inst) {
        with = std::max(with, col_lds_bytes(h, I, c.tk, true));
        without = std::max(without, col_lds_bytes(h, I, c.tk, false));
    }
    const int regs = h->dtype == LLG_F32 ? col_conv_vgprs<float>(h->max_nz, c.col_r)
                                         : col_conv_vgprs<double>(h->max_nz, c.col_r);
    return resident_blocks(with, regs, c.col_thr) >= resident_blocks(without, regs, c.col_thr);
}

// Likewise the forward row kernel stages the neighbour rows of y_s and psi in
// LDS only where that costs no resident block; otherwise it reads them from
// memory (wide rows: the 2048-point transforms already fill half the LDS).
bool fwd_stage_rows(const llg_handle* h, const LaunchCfg& c) {
    auto regs = [&](int staged) {
        return h->dtype == LLG_F32 ? stage_fwd_vgprs<float>(c.fwd_r, staged) : stage_fwd_vgprs<double>(c.fwd_r, staged);
    };
    return resident_blocks(loc_lds_bytes(h, 4), regs(1), c.fwd_thr) >=
           resident_blocks(loc_lds_bytes(h, 0), regs(0), c.fwd_thr);
}

int apply_cfg(llg_handle* h, const LaunchCfg& c) {
    const std::vector<int2> wc = column_work(h, c.tk);
    HIPCHK(hipMemcpy(h->work_col, wc.data(), wc.size() * sizeof(int2), hipMemcpyHostToDevice));
    const bool stage_tile = col_stage_tile(h, c);
    size_t col_lds = 0;
    for (auto& I : h->inst) col_lds = std::max(col_lds, col_lds_bytes(h, I, c.tk, stage_tile));
    const bool frows = fwd_stage_rows(h, c);
    const size_t loc_lds = loc_lds_bytes(h, 4), fwd_lds = loc_lds_bytes(h, frows ? 4 : 0),
                 bwd_lds = loc_lds_bytes(h, c.nv);
    auto fill = [&](auto& b) {
        b.ncol = (int)wc.size();
        b.col_tk = c.tk;
        b.col_threads = c.col_thr;
        b.col_radix = c.col_r;
        b.loc_threads = c.fwd_thr;
        b.loc_radix = c.fwd_r;
        b.bwd_threads = c.bwd_thr;
        b.bwd_radix = c.bwd_r;
        b.loc_nv = c.nv;
        b.loc_lds = loc_lds;
        b.fwd_lds = fwd_lds;
        b.fwd_rows = frows ? 1 : 0;
        b.bwd_lds = bwd_lds;
        b.col_lds = col_lds;
    };
    fill(h->bf);
    fill(h->bd);
    h->bf.col_nt_lds = h->bd.col_nt_lds = stage_tile ? 1 : 0;
    const size_t need = std::max(std::max(loc_lds, bwd_lds), col_lds);
    if (need > 65536) {
        hipError_t e = h->dtype == LLG_F32 ? set_lds_limits<float>(need) : set_lds_limits<double>(need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(LLG_ESHAPE, "kernels need " + std::to_string(need) + " bytes of LDS: " + hipGetErrorString(e));
        }
    }
    return LLG_OK;
}

int choose_launch(llg_handle* h) {
    // work lists: row pairs (fixed) and column tiles (capacity for the narrowest tile)
    std::vector<int2> wl;
    size_t ncol_max = 0;
    for (int i = 0; i < (int)h->inst.size(); ++i) {
        for (int r = 0; r < h->inst[i].nloc; ++r) wl.push_back(make_int2(i, r));
        ncol_max += (size_t)h->inst[i].ktiles * spec_tile_of((int)h->tsz);
    }
    ncol_max += (size_t)8 * spec_tile_of((int)h->tsz);  // empty items of the last group
    int rc;
    void* p;
    if ((rc = alloc(h, &p, wl.size() * sizeof(int2)))) return rc;
    h->work_loc = (int2*)p;
    HIPCHK(hipMemcpy(p, wl.data(), wl.size() * sizeof(int2), hipMemcpyHostToDevice));
    if ((rc = alloc(h, &p, ncol_max * sizeof(int2)))) return rc;
    h->work_col = (int2*)p;
    int max_n3 = 0;
    for (auto& I : h->inst) max_n3 = std::max(max_n3, 3 * I.N);
    auto fill = [&](auto& b) {
        b.work_loc = h->work_loc;
        b.work_col = h->work_col;
        b.nloc = (int)wl.size();
        b.ninst = (int)h->inst.size();
        b.max_n3 = max_n3;
    };
    fill(h->bf);
    fill(h->bd);
    LaunchCfg c;
    if ((rc = default_cfg(h, c))) return rc;
    return apply_cfg(h, c);
}

int validate_problem(const llg_problem* p) {
    if (!p) return fail(LLG_EINVAL, "problem is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LLG_EINVAL, "grid extents must be >= 1");
    if ((long long)p->nx * p->ny * p->nz > (1LL << 28)) return fail(LLG_ESHAPE, "grid too large");
    if (!(p->dx > 0 && p->dy > 0 && p->dz > 0)) return fail(LLG_EINVAL, "cell sizes must be > 0");
    if (!(p->Ms > 0)) return fail(LLG_EINVAL, "Ms must be > 0");
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(LLG_EINVAL, "dt must be finite and > 0");
    if (!(p->gamma > 0)) return fail(LLG_EINVAL, "gamma must be > 0");
    if (!(p->alpha0 >= 0) || !(p->alpha_max >= 0)) return fail(LLG_EINVAL, "damping must be >= 0");
    if (p->ramp_cells < 0) return fail(LLG_EINVAL, "ramp_cells must be >= 0");
    if (p->dtype != LLG_F32 && p->dtype != LLG_F64) return fail(LLG_EINVAL, "dtype must be LLG_F32 or LLG_F64");
    if (p->terms & ~15) return fail(LLG_EINVAL, "unknown term bits");
    if (p->nz > 8) return fail(LLG_ESHAPE, "nz > 8 is not supported by the column FFT");
    if (p->max_steps < 1) return fail(LLG_EINVAL, "max_steps must be >= 1");
    if (p->ckpt_policy != LLG_CKPT_SQRT && p->ckpt_policy != LLG_CKPT_ALL && p->ckpt_policy != LLG_CKPT_BINOMIAL)
        return fail(LLG_EINVAL, "unknown checkpoint policy");
    if (p->ckpt_param < 0) return fail(LLG_EINVAL, "ckpt_param must be >= 0");
    const double* vals[] = {&p->A, &p->K, &p->f1, &p->f2, &p->t_switch, &p->t_ramp};
    for (auto v : vals)
        if (!std::isfinite(*v)) return fail(LLG_EINVAL, "non-finite parameter");
    if (p->drive_kind != LLG_DRIVE_SINE && p->drive_kind != LLG_DRIVE_RAMP) return fail(LLG_EINVAL, "unknown drive kind");
    if (p->drive_kind == LLG_DRIVE_RAMP && !(p->t_ramp > 0)) return fail(LLG_EINVAL, "t_ramp must be > 0");
    if (!(p->psi_freeze >= 0 && p->psi_freeze < 1)) return fail(LLG_EINVAL, "psi_freeze must lie in [0, 1)");
    return LLG_OK;
}

// Arrays of 3N in the state buffer and in each snapshot: a float state is kept
// as hi + lo (the low part carries what rounding hi to float dropped).
int state_mult(const llg_handle* h) { return h->dtype == LLG_F32 ? 2 : 1; }

int take_events(llg_handle* h, hipEvent_t* a, hipEvent_t* b) {
    for (hipEvent_t* e : {a, b}) {
        if (!h->ev_pool.empty()) {
            *e = h->ev_pool.back();
            h->ev_pool.pop_back();
        } else {
            HIPCHK(hipEventCreate(e));
        }
    }
    return LLG_OK;
}

// move finished profiling records into the per-kind totals
int drain_profile(llg_handle* h) {
    for (auto& r : h->prof) {
        HIPCHK(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        h->prof_ms[r.kind] += ms;
        h->prof_bytes[r.kind] += r.bytes;
        h->prof_n[r.kind] += 1;
        h->ev_pool.push_back(r.a);
        h->ev_pool.push_back(r.b);
    }
    h->prof.clear();
    return LLG_OK;
}

// Binomial schedule for a run of n steps (kept until n or the slot count changes).
void ensure_plan(llg_handle* h, int64_t n) {
    if (h->policy != LLG_CKPT_BINOMIAL) return;
    const int slots = binomial_slots(n, h->ckpt_param);
    if (h->plan_n == n && h->plan_slots == slots) return;
    binomial_plan(n, slots, h->plan);
    h->plan_n = n;
    h->plan_slots = slots;
}

// What llg_adjoint needs to know about the last forward run.
void record_forward(llg_handle* h, double t0, int64_t n, const llg_objective_spec* obj) {
    h->fwd_valid = true;
    h->t0 = t0;
    h->n_steps = n;
    h->K_used = segment_length(n, h->policy, h->ckpt_param);
    h->last_obj = obj ? *obj : llg_objective_spec{};
    h->last_obj.freqs = h->last_obj.coef = nullptr;  // the caller's arrays are not kept
    h->last_obj.target = h->last_obj.weight = nullptr;
}

// Second stream and events of the overlapped adjoint (created outside any capture).
int prepare_adjoint(llg_handle* h) {
    if (h->policy == LLG_CKPT_BINOMIAL || h->halves < 2) return LLG_OK;
    const int64_t nseg = (h->n_steps + h->K_used - 1) / h->K_used;
    if (!h->aux) HIPCHK(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    while (h->sync_ev.size() < (size_t)(2 * nseg + 1)) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->sync_ev.push_back(e);
    }
    return LLG_OK;
}

void drop_graphs(llg_handle* h) {
    for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

// Run body(stream) -- an enqueue-only launch sequence whose kernels touch only
// handle buffers -- either directly on s or, with graphs enabled, as a cached
// HIP graph on the handle's graph stream, ordered after s's prior work and
// before its later work.  body returns an int status and sets *result.
// Sequences of more than kGraphMaxSteps RK4 steps run directly: graphs of
// that length (~10^5 nodes) are not supported.
constexpr int64_t kGraphMaxSteps = 2000;

template <typename F>
int run_sequence(llg_handle* h, hipStream_t s, const std::vector<double>& key, int64_t n_steps, int* result,
                 F&& body) {
    if (!h->graphs_on || h->prof_on || n_steps > kGraphMaxSteps) return body(s, result);
    if (!h->gstream) {
        HIPCHK(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&h->g_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->g_out, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(h->g_in, s));
    HIPCHK(hipStreamWaitEvent(h->gstream, h->g_in, 0));
    llg_handle::GraphEntry* hit = nullptr;
    for (auto& g : h->graphs)
        if (g.key == key) hit = &g;
    if (!hit) {
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
        int res = 0;
        const int rc = body(h->gstream, &res);
        const hipError_t e = hipStreamEndCapture(h->gstream, &graph);
        if (rc) {
            if (e == hipSuccess && graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(LLG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(LLG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
        if (h->graphs.size() >= 8) {
            (void)hipGraphExecDestroy(h->graphs.front().exec);
            h->graphs.erase(h->graphs.begin());
        }
        h->graphs.push_back({key, exec, res});
        hit = &h->graphs.back();
    }
    *result = hit->result;
    HIPCHK(hipGraphLaunch(hit->exec, h->gstream));
    HIPCHK(hipEventRecord(h->g_out, h->gstream));
    HIPCHK(hipStreamWaitEvent(s, h->g_out, 0));
    return LLG_OK;
}

// ---------------------------------------------------------------------------
// typed orchestration (all instances of the batch at once)
// ---------------------------------------------------------------------------
template <typename T>
struct Ops {
    using C = cplx<T>;
    llg_handle* h;
    hipStream_t s;
    int adj_lambda0 = B_L0;
    int spec = B_S;  // x-spectrum buffer of this stream's forward work
    // adjoint state: ping-pong roles of lambda and u, port window
    int Lc = B_L0, Lo = B_L1, Uc = B_U0, Uo = B_U1;
    bool adj_port = false;
    bool adj_spec = false;
    bool adj_curve = false;
    int64_t adj_nstart = 0;
    int adj_W = 0;
    const BatchDev<T>& B() const { return bdev<T>(h); }

    // every kernel launch goes through here: optional event bracketing for profiling
    // every kernel launch goes through here.  Profiling binds an event pair to
    // the dispatch of the three per-stage kernels (device start/end of the
    // kernel itself, not of the surrounding queue activity).
    template <typename F>
    int run(int kind, double bytes, F&& launch) {
        hipEvent_t a = nullptr, b = nullptr;
        const bool rec = h->prof_on && kind >= 0 && (h->prof_seen[kind]++ % h->prof_stride) == 0;
        if (rec)
            if (int rc = take_events(h, &a, &b)) return rc;
        hipError_t e = launch(a, b);
        if (e != hipSuccess) return fail(LLG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
        if (rec) h->prof.push_back({kind, bytes, a, b});
        return LLG_OK;
    }

    // algorithmic HBM bytes of one launch over the batch (each element read or written once)
    double fwd_bytes(const FwdL& L) const {
        const double t = sizeof(T), n = h->sumN;
        double b = n * 4 * t;  // ys, psi
        if (L.do_inv) b += h->sumSpec;
        if (L.do_fwd) b += h->sumSpec;
        switch (L.stage) {
            case 0: b += n * 6 * t; break;
            case 1: case 2: b += n * 12 * t; break;
            case 3: b += n * (state_mult(h) > 1 ? 15 : 9) * t; break;  // + lo r/w of a float state
            case -1: b += n * 3 * t * (L.ext_ynext ? 2 : 1); break;
            default: break;
        }
        if (L.store_j >= 0) b += n * 6 * t;
        if (L.port) b += 2 * n;
        return b;
    }
    double bwd_bytes(const BwdL& L) const {
        const double t = sizeof(T), n = h->sumN;
        double b;
        if (L.stage < 0) {
            b = n * 13 * t + h->sumSpec;
        } else {
            b = n * (16 * t + 16) + (L.stage == 3 || L.ext_lacc ? 0 : n * 3 * t);
            if (L.prev_j >= 0) b += n * 9 * t;
            if (L.do_inv) b += h->sumSpec;
            if (L.do_fwd) b += h->sumSpec;
            if (L.port_src) b += 2 * n;
        }
        return b;
    }
    double col_bytes() const { return 2 * h->sumSpec + h->sumNhat; }

    int col() {
        if (!h->demag) return LLG_OK;
        return run(LLG_KIND_COLUMN, col_bytes(), [&](hipEvent_t a, hipEvent_t b) { return launch_col_conv<T>(B(), h->max_nz, spec, s, a, b); });
    }
    int fwd(const FwdL& L) {
        return run(LLG_KIND_STAGE_FWD, fwd_bytes(L), [&](hipEvent_t a, hipEvent_t b) { return launch_stage_fwd<T>(B(), L, s, a, b); });
    }
    int bwd(const BwdL& L) {
        return run(LLG_KIND_STAGE_BWD, bwd_bytes(L), [&](hipEvent_t a, hipEvent_t b) { return launch_stage_bwd<T>(B(), L, s, a, b); });
    }
    // copies of the state m_n to and from the snapshots; a float state is hi + lo (twice 3N)
    int copy(int src, int src_slot, int dst, int dst_slot) {
        const int mult = state_mult(h);
        return run(-1, 0, [&](hipEvent_t, hipEvent_t) {
            return launch_copy<T>(B(), src, src_slot, dst, dst_slot, mult, s);
        });
    }

    FwdL fwd_launch(int stage) const {
        FwdL L{};
        L.stage = stage;
        L.ys = L.mn = L.acc = L.ynext = -1;
        L.store_j = -1;
        L.spec = spec;
        return L;
    }

    // spectrum of psi * m into S
    int prologue(void* ext_m = nullptr) {
        if (!h->demag) return LLG_OK;
        FwdL L = fwd_launch(-3);
        L.ys = B_M;
        L.ext_ys = ext_m;
        L.do_fwd = 1;
        return fwd(L);
    }

    // one RK4 step from B_M (spectrum of psi*m already in S); optional stage store
    // port: 0 none, 1 accumulate the m_y^2 sums, 2 store the m_y sums of window step pstep
    int step(double t, bool last, int store_j, int port, int pstep = -1) {
        const double dt = h->inst[0].prob.dt;
        const double cs[4] = {0.0, 0.5, 0.5, 1.0};
        const int y_in[4] = {B_M, B_YA, B_YB, B_YA};
        const int y_out[4] = {B_YA, B_YB, B_YA, B_M};
        for (int st = 0; st < 4; ++st) {
            if (int rc = col()) return rc;
            FwdL L = fwd_launch(st);
            L.t = t + cs[st] * dt;
            L.ys = y_in[st];
            L.mn = B_M;
            L.acc = B_ACC;
            L.ynext = y_out[st];
            L.store_j = store_j;
            L.port = st == 3 ? port : 0;
            L.pstep = pstep;
            L.do_inv = h->demag;
            L.do_fwd = h->demag && !(last && st == 3);
            if (int rc = fwd(L)) return rc;
        }
        return LLG_OK;
    }

    int forward(double t0, int64_t n, const llg_objective_spec* obj) {
        const bool spec = obj && obj->kind == LLG_OBJ_PORT_SPECTRAL;
        const bool curve = obj && obj->kind == LLG_OBJ_MAG_CURVE;
        const bool port = obj && (obj->kind == LLG_OBJ_PORT_MY2 || spec || curve);
        const double dt = h->inst[0].prob.dt;
        // port mode of step k (which produces m_{k+1}) and its window index
        const int mode = curve ? 3 : (spec ? 2 : 1);
        auto in_win = [&](int64_t k) { return port && (k + 1) > obj->n_start ? mode : 0; };
        auto wstep = [&](int64_t k) { return port ? (int)(k - obj->n_start) : -1; };
        const int64_t K = segment_length(n, h->policy, h->ckpt_param);
        if (h->policy == LLG_CKPT_BINOMIAL) {
            if (binomial_slots(n, h->ckpt_param) > h->nsnap)
                return fail(LLG_ENOMEM, "checkpoint store too small for n_steps (raise max_steps at create)");
        } else if ((n + K - 1) / K > h->nsnap || K > h->K) {
            return fail(LLG_ENOMEM, "checkpoint store too small for n_steps (raise max_steps at create)");
        }
        if (mode == 1 && port)
            if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_zero<T>(B(), B_PPART, 1, s); })) return rc;
        if (state_mult(h) > 1)  // the caller's m0 is a float state: its low part is zero
            if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_fill<T>(B(), B_M, 3, 0.0, s, 3); }))
                return rc;
        if (int rc = prologue()) return rc;
        int64_t k = 0;
        if (h->policy == LLG_CKPT_BINOMIAL) {
            // the forward part of the binomial schedule: snapshots along its first descent
            ensure_plan(h, n);
            if (int rc = copy(B_M, 0, B_SNAP, 0)) return rc;
            for (size_t a = 0; a < h->plan.split; ++a) {
                const PlanAct& q = h->plan.acts[a];
                if (q.op == P_LOAD && q.a != k) return fail(LLG_ESTATE, "internal error: checkpoint schedule");
                if (q.op == P_ADV) {
                    if (q.a != k) return fail(LLG_ESTATE, "internal error: checkpoint schedule");
                    for (; k < q.b; ++k)
                        if (int rc = step(t0 + (double)k * dt, k == n - 1, -1, in_win(k), wstep(k))) return rc;
                }
                if (q.op == P_SAVE)
                    if (int rc = copy(B_M, 0, B_SNAP, q.slot)) return rc;
            }
        }
        for (; k < n; ++k) {
            if (h->policy != LLG_CKPT_BINOMIAL && k % K == 0)
                if (int rc = copy(B_M, 0, B_SNAP, (int)(k / K))) return rc;
            if (int rc = step(t0 + (double)k * dt, k == n - 1, -1, in_win(k), wstep(k))) return rc;
        }
        if (port) {
            const int W = (int)(n - obj->n_start);
            if (curve) {
                if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_curve<T>(B(), h->curve_tw, W, s); }))
                    return rc;
            } else if (spec) {
                if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) {
                        return launch_spectral<T>(B(), h->spec_fc, obj->n_freq, W, t0, obj->n_start, dt, s);
                    }))
                    return rc;
            } else if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_port_finish<T>(B(), W, s); })) {
                return rc;
            }
        }
        h->fwd_valid = true;
        h->t0 = t0;
        h->n_steps = n;
        h->K_used = K;
        h->last_obj = obj ? *obj : llg_objective_spec{};
        return LLG_OK;
    }

    int field(const void* m, double t, void* Bout, void* rhs) {
        if (int rc = prologue(const_cast<void*>(m))) return rc;
        if (int rc = col()) return rc;
        FwdL L = fwd_launch(-1);
        L.t = t;
        L.ys = B_M;
        L.ext_ys = const_cast<void*>(m);
        L.ext_ynext = rhs;
        L.ext_B = Bout;
        L.do_inv = h->demag;
        return fwd(L);
    }

    // ---- adaptive Dormand-Prince 5(4) (single instance) -------------------
    static constexpr double kC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
    static constexpr double kA[7][6] = {{0, 0, 0, 0, 0, 0},
                                        {1.0 / 5, 0, 0, 0, 0, 0},
                                        {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
                                        {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
                                        {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
                                        {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
                                        {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
    static constexpr double kB5[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
    static constexpr double kB4[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200,
                                      187.0 / 2100, 1.0 / 40};

    T* P(void* v) const { return static_cast<T*>(v); }
    size_t n3() const { return (size_t)3 * h->inst[0].N; }
    T* slot(int id, int j) const { return static_cast<T*>(h->inst[0].tab.b[id]) + (size_t)j * 4 * n3(); }
    // stage st of a step from m at (t, hstep): Y = m + hstep sum_j a_st,j k_j, rate k_st = f(Y, t + c_st hstep)
    int dp_stage(int st, const T* m, double t, double hstep, T* Y, void* Bout) {
        const auto& D = h->dp;
        const T* y = m;
        if (st > 0) {
            LinTerms<T> lt{};
            for (int j = 0; j < st; ++j)
                if (kA[st][j] != 0.0) {
                    lt.src[lt.nt] = P(D.k[j]);
                    lt.c[lt.nt] = hstep * kA[st][j];
                    ++lt.nt;
                }
            if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_lincomb<T>((int)n3(), Y, m, lt, s); }))
                return rc;
            y = Y;
        } else if (Y != m) {
            HIPCHK(hipMemcpyAsync(Y, m, n3() * sizeof(T), hipMemcpyDeviceToDevice, s));
            y = Y;
        }
        return field(y, t + kC[st] * hstep, Bout, D.k[st]);
    }

    // Trial step from m: y5 and the error norm (device double at D.err[0]).
    // Stage store of step n: the field of stage s (s = 0..5) and the state of stage s (s = 1..5).
    T* kept_B(int64_t n, int st) const { return P(h->dp.stages) + ((size_t)n * 11 + (st ? 2 * st : 0)) * n3(); }
    T* kept_Y(int64_t n, int st) const { return P(h->dp.stages) + ((size_t)n * 11 + 2 * st - 1) * n3(); }

    // One trial step.  Stage s's field evaluation also forms stage s + 1's state (the stage-sum variant of the
    // forward kernel: the rate it computes enters last, after the earlier rates, in the order and with the fused
    // multiply-adds of the stage-sum kernel) and transforms it for the next column pass, so that a stage costs
    // two launches.  The last stage's state is y5 itself (its coefficients are the fifth-order weights) and its
    // time is t + h: the rate there, k[6], is the next step's k[0] (first same as last).  With have_k0, k[0]
    // already holds f(m, t).  With the stage store, trial step n writes its stage states and fields into slot n
    // (a rejected trial's are overwritten by the next) and the field at y5 into slot n + 1 as that step's
    // stage-0 field.
    int dp_trial(int64_t n, const T* m, double t, double hstep, double rtol, double atol, bool have_k0) {
        auto& D = h->dp;
        const bool keep = D.keep;
        if (!have_k0)
            if (int rc = dp_stage(0, m, t, hstep, P(D.ystage), keep ? kept_B(n, 0) : nullptr)) return rc;
        T* Y = keep ? kept_Y(n, 1) : P(D.ystage);
        {
            LinTerms<T> lt{};
            lt.src[0] = P(D.k[0]);
            lt.c[0] = hstep * kA[1][0];
            lt.nt = 1;
            if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_lincomb<T>((int)n3(), Y, m, lt, s); }))
                return rc;
        }
        if (int rc = prologue(Y)) return rc;
        for (int st = 1; st < 6; ++st) {
            T* Yn = st == 5 ? P(D.y5) : keep ? kept_Y(n, st + 1) : (Y == P(D.ystage) ? P(D.ystage2) : P(D.ystage));
            if (int rc = col()) return rc;
            FwdL L = fwd_launch(-1);
            L.t = t + kC[st] * hstep;
            L.ys = B_M;
            L.ext_ys = Y;
            L.ext_ynext = D.k[st];
            L.ext_B = keep ? kept_B(n, st) : nullptr;
            L.do_inv = h->demag;
            L.do_fwd = h->demag;
            L.lin_base = m;
            for (int j = 0; j < st; ++j)
                if (kA[st + 1][j] != 0.0) {
                    L.lin_src[L.lin_nt] = D.k[j];
                    L.lin_c[L.lin_nt++] = hstep * kA[st + 1][j];
                }
            L.lin_cf = hstep * kA[st + 1][st];
            L.lin_out = Yn;
            if (int rc = fwd(L)) return rc;
            Y = Yn;
        }
        {
            // the rate at y5 (its spectrum is in S)
            if (int rc = col()) return rc;
            FwdL L = fwd_launch(-1);
            L.t = t + kC[6] * hstep;
            L.ys = B_M;
            L.ext_ys = D.y5;
            L.ext_ynext = D.k[6];
            L.ext_B = keep ? kept_B(n + 1, 0) : nullptr;
            L.do_inv = h->demag;
            if (int rc = fwd(L)) return rc;
        }
        LinTerms<T> e{};
        for (int j = 0; j < 7; ++j) {
            e.src[e.nt] = P(D.k[j]);
            e.c[e.nt] = hstep * (kB5[j] - kB4[j]);
            ++e.nt;
        }
        return run(-1, 0, [&](hipEvent_t, hipEvent_t) {
            return launch_err_norm<T>((int)n3(), m, P(D.y5), e, rtol, atol, D.err + 8, D.err, s);
        });
    }

    // mu = J_f(Y)^T kappa for the state Y with field Bf = B(Y) and kappa = sum_q kap.c[q] kap.src[q], formed by
    // the seed launch: the field adjoint u and its spectrum, the column pass, then the transpose (stage 0 without
    // a next stage), written to mu_out; dJ/dpsi gains kappa . df/dpsi(Y).  Y and Bf are read where they are.
    int stage_transpose(const T* Y, const T* Bf, const LinTerms<T>& kap, void* mu_out) {
        BwdL Ls{};
        Ls.stage = -2;
        Ls.seed_unit = 1;
        for (int q = 0; q < kap.nt; ++q) {
            Ls.lin_src[q] = kap.src[q];
            Ls.lin_c[q] = kap.c[q];
        }
        Ls.lin_nt = kap.nt;
        Ls.j = Ls.prev_j = 0;
        Ls.prev_st = 0;
        Ls.ucur = -1;
        Ls.unext = B_U0;
        Ls.lamp = B_L0;
        Ls.lacc = -1;
        Ls.do_fwd = h->demag;
        Ls.ext_ys = const_cast<T*>(Y);
        if (int rc = bwd(Ls)) return rc;
        if (int rc = col()) return rc;
        BwdL Lf{};
        Lf.stage = 0;
        Lf.j = 0;
        Lf.prev_j = -1;
        Lf.prev_st = 3;
        Lf.ucur = B_U0;
        Lf.unext = B_U1;
        Lf.lamp = B_L0;
        Lf.lacc = -1;
        Lf.do_inv = h->demag;
        Lf.do_fwd = 0;
        Lf.ext_ys = const_cast<T*>(Y);
        Lf.ext_B = const_cast<T*>(Bf);
        Lf.ext_lacc = mu_out;
        return bwd(Lf);
    }
    static LinTerms<T> kappa(std::initializer_list<std::pair<double, const void*>> terms) {
        LinTerms<T> lt{};
        for (auto& tm : terms) {
            lt.src[lt.nt] = static_cast<const T*>(tm.second);
            lt.c[lt.nt++] = tm.first;
        }
        return lt;
    }

    // Cubic Hermite interpolant of the kept states on [t_n, t_n + h] at t_n + th h into Y:
    // h00 m_n + h10 h f(m_n) + h01 m_n+1 + h11 h f(m_n+1), with f(m_n) in k[1] and f(m_n+1) in k[0].
    int hermite(const T* m0, const T* m1, double hstep, double th, T* Y) {
        const auto& D = h->dp;
        LinTerms<T> lt{};
        const double th2 = th * th, th3 = th2 * th;
        lt.src[0] = m0;
        lt.c[0] = 2.0 * th3 - 3.0 * th2 + 1.0;
        lt.src[1] = P(D.k[1]);
        lt.c[1] = (th3 - 2.0 * th2 + th) * hstep;
        lt.src[2] = m1;
        lt.c[2] = 3.0 * th2 - 2.0 * th3;
        lt.src[3] = P(D.k[0]);
        lt.c[3] = (th3 - th2) * hstep;
        lt.nt = 4;
        return run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_lincomb<T>((int)n3(), Y, nullptr, lt, s); });
    }

    // Continuous adjoint (Eqs. 6-7) over the kept states of the last adaptive run: each interval is split into
    // n_sub classic RK4 steps backwards for the augmented system (a, dJ/dpsi), with the Jacobians at the
    // sub-step's end, the Hermite state at its midpoint (twice) and its start.  Stage slots of YS / BS:
    // 0 and 2 alternate as the sub-step's end and start, 1 = midpoint, 3 = m_n.
    int continuous_adjoint(bool use_expl, int n_sub) {
        auto& D = h->dp;
        const size_t nb = n3() * sizeof(T);
        if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_zero<T>(B(), B_GPSI, 0, s); })) return rc;
        const int64_t N = (int64_t)D.hs.size();
        const T* snaps = P(D.snaps);
        const double tN = D.ts.empty() ? 0.0 : D.ts.back() + D.hs.back();
        HIPCHK(hipMemcpyAsync(slot(B_YS, 0), snaps + (size_t)N * n3(), nb, hipMemcpyDeviceToDevice, s));
        if (int rc = field(slot(B_YS, 0), tN, slot(B_BS, 0), D.k[0])) return rc;
        for (int64_t n = N - 1; n >= 0; --n) {
            const double hn = D.hs[n], t = D.ts[n], hsub = hn / n_sub;
            const T* m0 = snaps + (size_t)n * n3();
            const T* m1 = snaps + (size_t)(n + 1) * n3();
            HIPCHK(hipMemcpyAsync(slot(B_YS, 3), m0, nb, hipMemcpyDeviceToDevice, s));
            if (int rc = field(slot(B_YS, 3), t, slot(B_BS, 3), D.k[1])) return rc;
            int up = 0;
            for (int k = n_sub - 1; k >= 0; --k) {
                const double thm = (k + 0.5) / n_sub;
                if (int rc = hermite(m0, m1, hn, thm, slot(B_YS, 1))) return rc;
                if (int rc = field(slot(B_YS, 1), t + thm * hn, slot(B_BS, 1), D.k[2])) return rc;
                int lo = 3;
                if (k > 0) {
                    lo = up == 0 ? 2 : 0;
                    const double thl = (double)k / n_sub;
                    if (int rc = hermite(m0, m1, hn, thl, slot(B_YS, lo))) return rc;
                    if (int rc = field(slot(B_YS, lo), t + thl * hn, slot(B_BS, lo), D.k[2])) return rc;
                }
                // kappa_s = w_s hsub A_s gives mu_s = w_s hsub G_s: A2 = a + 3 mu1, A3 = a + 1.5 mu2,
                // A4 = a + 3 mu3, and a <- a + mu1 + mu2 + mu3 + mu4
                if (int rc = stage_transpose(slot(B_YS, up), slot(B_BS, up), kappa({{hsub / 6.0, D.lam}}), D.mu[0]))
                    return rc;
                if (int rc = stage_transpose(slot(B_YS, 1), slot(B_BS, 1), kappa({{hsub / 3.0, D.lam}, {hsub, D.mu[0]}}),
                                             D.mu[1]))
                    return rc;
                if (int rc = stage_transpose(slot(B_YS, 1), slot(B_BS, 1),
                                             kappa({{hsub / 3.0, D.lam}, {hsub / 2.0, D.mu[1]}}), D.mu[2]))
                    return rc;
                if (int rc = stage_transpose(slot(B_YS, lo), slot(B_BS, lo),
                                             kappa({{hsub / 6.0, D.lam}, {hsub / 2.0, D.mu[2]}}), D.mu[3]))
                    return rc;
                LinTerms<T> lt{};
                for (int q = 0; q < 4; ++q) {
                    lt.src[q] = P(D.mu[q]);
                    lt.c[q] = 1.0;
                }
                lt.nt = 4;
                if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_lincomb<T>((int)n3(), P(D.ystage), P(D.lam), lt, s); }))
                    return rc;
                HIPCHK(hipMemcpyAsync(D.lam, D.ystage, nb, hipMemcpyDeviceToDevice, s));
                up = lo;
            }
            // m_n and its field and rate become the next interval's end
            HIPCHK(hipMemcpyAsync(slot(B_YS, 0), slot(B_YS, 3), nb, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(slot(B_BS, 0), slot(B_BS, 3), nb, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(D.k[0], D.k[1], nb, hipMemcpyDeviceToDevice, s));
        }
        return run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_psi_grad_out<T>(B(), use_expl, s); });
    }

    // Discrete adjoint of the accepted steps (sizes fixed), from lambda_N in D.lam.
    int dp_adjoint(bool use_expl) {
        auto& D = h->dp;
        const size_t nb = n3() * sizeof(T);
        if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_zero<T>(B(), B_GPSI, 0, s); })) return rc;
        for (int64_t n = (int64_t)D.hs.size() - 1; n >= 0; --n) {
            const double hstep = D.hs[n], t = D.ts[n];
            const T* m = P(D.snaps) + (size_t)n * n3();
            // the stages this step's transpose needs (the 7th has b = 0 and feeds no stage): read in the stage
            // store when the forward filled it, else recomputed from the kept state (bitwise the same values)
            const T* Ys[6];
            const T* Bs[6];
            if (D.stages_valid) {
                for (int st = 0; st < 6; ++st) {
                    Ys[st] = st ? kept_Y(n, st) : m;
                    Bs[st] = kept_B(n, st);
                }
            } else {
                for (int st = 0; st < 6; ++st) {
                    if (int rc = dp_stage(st, m, t, hstep, slot(B_YS, st), slot(B_BS, st))) return rc;
                    Ys[st] = slot(B_YS, st);
                    Bs[st] = slot(B_BS, st);
                }
            }
            for (int st = 5; st >= 0; --st) {
                // kappa_s = h (b_s lambda' + sum_{i>s} a_is mu_i), formed by the transpose's seed launch
                LinTerms<T> lt{};
                lt.src[lt.nt] = P(D.lam);
                lt.c[lt.nt++] = hstep * kB5[st];
                for (int i = st + 1; i < 6; ++i)
                    if (kA[i][st] != 0.0) {
                        lt.src[lt.nt] = P(D.mu[i]);
                        lt.c[lt.nt++] = hstep * kA[i][st];
                    }
                if (int rc = stage_transpose(Ys[st], Bs[st], lt, D.mu[st])) return rc;
            }
            // lambda_n = lambda' + sum_s mu_s
            LinTerms<T> lt{};
            for (int st = 0; st < 6; ++st) {
                lt.src[lt.nt] = P(D.mu[st]);
                lt.c[lt.nt++] = 1.0;
            }
            if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_lincomb<T>((int)n3(), P(D.ystage), P(D.lam), lt, s); }))
                return rc;
            HIPCHK(hipMemcpyAsync(D.lam, D.ystage, nb, hipMemcpyDeviceToDevice, s));
        }
        return run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_psi_grad_out<T>(B(), use_expl, s); });
    }

    int energy(const llg_objective_spec* obj, const T* m, double t, double* J, T* dJdm, double* dJdpsi, double* en) {
        if (int rc = prologue(const_cast<T*>(m))) return rc;
        if (int rc = col()) return rc;
        const llg_problem& q = h->inst[0].prob;
        const double MsV = q.Ms * q.dx * q.dy * q.dz;
        if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_energy<T>(B(), t, m, MsV / obj->E_ref, dJdm, dJdpsi, s); }))
            return rc;
        return run(-1, 0, [&](hipEvent_t, hipEvent_t) {
            return launch_energy_finish<T>(B(), MsV, obj->lambda, obj->area, obj->E_ref, J, en, dJdpsi, s);
        });
    }

    // Recompute steps [n0, n1) from m_{n0} (in B_M), storing the stage states
    // and fields of step k in stage slot off + k - n0.
    int recompute(int64_t n0, int64_t n1, int off) {
        const double dt = h->inst[0].prob.dt;
        if (int rc = prologue()) return rc;
        for (int64_t k = n0; k < n1; ++k)
            if (int rc = step(h->t0 + (double)k * dt, k == n1 - 1, off + (int)(k - n0), 0)) return rc;
        return LLG_OK;
    }

    // Transpose steps n1-1 .. n0, whose stage states sit in slots off .. off + n1 - n0 - 1.
    int backward(int64_t n0, int64_t n1, int off) {
        {
            // seed: l_4 and u_4 of the last step of the range
            BwdL L{};
            L.stage = -2;
            L.j = L.prev_j = off + (int)(n1 - 1 - n0);
            L.prev_st = 3;
            L.ucur = -1;
            L.unext = Uc;
            L.lamp = Lc;
            L.lacc = -1;
            L.do_fwd = h->demag;
            if (int rc = bwd(L)) return rc;
        }
        for (int64_t k = n1 - 1; k >= n0; --k) {
            const int j = off + (int)(k - n0);
            for (int st = 3; st >= 0; --st) {
                if (int rc = col()) return rc;
                BwdL L{};
                L.stage = st;
                L.j = j;
                L.prev_j = st > 0 ? j : (k > n0 ? j - 1 : -1);
                L.prev_st = st > 0 ? st - 1 : 3;
                L.ucur = Uc;
                L.unext = Uo;
                L.lamp = Lc;
                L.lacc = Lo;
                L.port_src = st == 0 && adj_port && k > adj_nstart;
                L.W = adj_W;
                L.port_lin = adj_curve ? 2 : (adj_spec ? 1 : 0);
                L.pstep = (int)(k - adj_nstart - 1);
                L.do_inv = h->demag;
                L.do_fwd = h->demag && L.prev_j >= 0;
                if (int rc = bwd(L)) return rc;
                if (L.prev_j >= 0) std::swap(Uc, Uo);
            }
            std::swap(Lc, Lo);  // lambda_k is the lambda' of step k-1
        }
        return LLG_OK;
    }


    int adjoint(const llg_objective_spec* obj, bool use_djdm, bool use_expl) {
        if (!h->fwd_valid) return fail(LLG_ESTATE, "llg_adjoint needs a preceding llg_forward on this handle");
        const int64_t n = h->n_steps, K = h->K_used;
        const double dt = h->inst[0].prob.dt;
        adj_spec = obj && obj->kind == LLG_OBJ_PORT_SPECTRAL;
        adj_curve = obj && obj->kind == LLG_OBJ_MAG_CURVE;
        adj_port = obj && (obj->kind == LLG_OBJ_PORT_MY2 || adj_spec || adj_curve);
        adj_nstart = adj_port ? obj->n_start : n;
        adj_W = (int)(n - adj_nstart);
        Lc = B_L0, Lo = B_L1, Uc = B_U0, Uo = B_U1;
        // dJ/dpsi starts at zero (the curve objective's terminal term adds to it);
        // lambda_N = dJ/dm_N (+ port source at N); B_M holds m_N
        if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_zero<T>(B(), B_GPSI, 0, s); })) return rc;
        const int port_mode = adj_port ? (adj_curve ? 3 : (adj_spec ? 2 : 1)) : 0;
        if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_adj_init<T>(B(), Lc, use_djdm, port_mode, adj_W, s); }))
            return rc;
        if (h->policy == LLG_CKPT_BINOMIAL) {
            // the rest of the binomial schedule, on this stream
            int64_t cur = n;
            for (size_t a = h->plan.split; a < h->plan.acts.size(); ++a) {
                const PlanAct& q = h->plan.acts[a];
                if (q.op == P_LOAD) {
                    if (cur != q.a) {
                        if (int rc = copy(B_SNAP, q.slot, B_M, 0)) return rc;
                        cur = q.a;
                    }
                } else if (q.op == P_ADV) {
                    if (cur != q.a) return fail(LLG_ESTATE, "internal error: checkpoint schedule");
                    if (int rc = prologue()) return rc;
                    for (int64_t k = q.a; k < q.b; ++k)
                        if (int rc = step(h->t0 + (double)k * dt, k == q.b - 1, -1, 0)) return rc;
                    cur = q.b;
                } else if (q.op == P_SAVE) {
                    if (int rc = copy(B_M, 0, B_SNAP, q.slot)) return rc;
                } else {
                    if (cur != q.a) return fail(LLG_ESTATE, "internal error: checkpoint schedule");
                    if (int rc = recompute(q.a, q.a + 1, 0)) return rc;
                    cur = q.a + 1;
                    if (int rc = backward(q.a, q.a + 1, 0)) return rc;
                }
            }
        } else {
            const int64_t nseg = (n + K - 1) / K;
            if (nseg == 1 || h->halves < 2) {
                for (int64_t seg = nseg - 1; seg >= 0; --seg) {
                    const int64_t n0 = seg * K, n1 = std::min(n, n0 + K);
                    if (int rc = copy(B_SNAP, (int)seg, B_M, 0)) return rc;
                    if (int rc = recompute(n0, n1, 0)) return rc;
                    if (int rc = backward(n0, n1, 0)) return rc;
                }
            } else {
                // segment seg-1 is recomputed on the second stream (own spectrum
                // buffer, other half of the stage store) while seg is transposed here
                if (!h->aux || h->sync_ev.size() < (size_t)(2 * nseg + 1))
                    return fail(LLG_ESTATE, "internal error: adjoint streams not prepared");
                hipEvent_t* ev_rec = h->sync_ev.data();
                hipEvent_t* ev_bwd = ev_rec + nseg;
                hipEvent_t ev_init = ev_rec[2 * nseg];
                Ops R{h, h->aux};
                R.spec = B_S2;
                HIPCHK(hipEventRecord(ev_init, s));
                HIPCHK(hipStreamWaitEvent(h->aux, ev_init, 0));
                auto rec = [&](int64_t seg) -> int {
                    const int64_t n0 = seg * K, n1 = std::min(n, n0 + K);
                    if (int rc = R.copy(B_SNAP, (int)seg, B_M, 0)) return rc;
                    if (int rc = R.recompute(n0, n1, (int)(K * (seg & 1)))) return rc;
                    HIPCHK(hipEventRecord(ev_rec[seg], h->aux));
                    return LLG_OK;
                };
                if (int rc = rec(nseg - 1)) return rc;
                for (int64_t seg = nseg - 1; seg >= 0; --seg) {
                    if (seg >= 1) {
                        // the half that seg-1 overwrites was last read by the transpose of seg+1
                        if (seg + 1 < nseg) HIPCHK(hipStreamWaitEvent(h->aux, ev_bwd[seg + 1], 0));
                        if (int rc = rec(seg - 1)) return rc;
                    }
                    HIPCHK(hipStreamWaitEvent(s, ev_rec[seg], 0));
                    const int64_t n0 = seg * K, n1 = std::min(n, n0 + K);
                    if (int rc = backward(n0, n1, (int)(K * (seg & 1)))) return rc;
                    HIPCHK(hipEventRecord(ev_bwd[seg], s));
                }
            }
        }
        if (int rc = run(-1, 0, [&](hipEvent_t, hipEvent_t) { return launch_psi_grad_out<T>(B(), use_expl, s); })) return rc;
        adj_lambda0 = Lc;
        return LLG_OK;
    }
};

// Autotuner: time the column kernel over the valid (tile, threads) pairs and
// the row kernels (one forward and one backward stage) over the valid block
// sizes, on the handle's own buffers (psi = 1, states zero), and keep the
// fastest.  Every candidate computes the same bits, so tuning changes speed only.
template <typename T>
int autotune_typed(llg_handle* h, hipStream_t s, LaunchCfg& best) {
    Ops<T> o{h, s};
    const size_t t = h->tsz;
    for (auto& I : h->inst) {
        const size_t n3 = (size_t)3 * I.N * t;
        for (int id : {B_M, B_ACC, B_YA, B_YB, B_ELL, B_U0, B_U1, B_L0, B_L1})
            HIPCHK(hipMemsetAsync(I.tab.b[id], 0, n3, s));
        HIPCHK(hipMemsetAsync(I.tab.b[B_YS], 0, 4 * n3, s));
        HIPCHK(hipMemsetAsync(I.tab.b[B_BS], 0, 4 * n3, s));
        HIPCHK(hipMemsetAsync(I.tab.b[B_GPSI], 0, (size_t)I.N * 8, s));
        if (h->demag) HIPCHK(hipMemsetAsync(I.tab.b[B_S], 0, (size_t)3 * I.nrows * I.Kx * 2 * t, s));
    }
    HIPCHK(launch_fill<T>(bdev<T>(h), B_PSI, 1, 1.0, s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int rc = LLG_OK;
    auto timed = [&](auto&& body) -> float {
        for (int k = 0; k < 2 && !rc; ++k) rc = body();
        if (rc || hipEventRecord(e0, s) != hipSuccess) return 1e30f;
        for (int k = 0; k < 8 && !rc; ++k) rc = body();
        float ms = 1e30f;
        if (rc || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return 1e30f;
        return ms;
    };
    FwdL Lf = o.fwd_launch(1);
    Lf.ys = B_YA;
    Lf.mn = B_M;
    Lf.acc = B_ACC;
    Lf.ynext = B_YB;
    Lf.do_inv = Lf.do_fwd = h->demag;
    BwdL Lb{};
    Lb.stage = 1;
    Lb.ucur = B_U0;
    Lb.unext = B_U1;
    Lb.lamp = B_L0;
    Lb.lacc = B_L1;
    Lb.do_inv = Lb.do_fwd = h->demag;
    LaunchCfg cur;
    if ((rc = default_cfg(h, cur))) return rc;
    best = cur;
    if (h->demag) {
        float tbest = 1e30f;
        for (int cr : {4, 8, 16}) {
            if (!radix_ok(h, cr)) continue;
            for (int tk : {1, 2, 4, 8, 16}) {
                if (tk > spec_tile_of((int)h->tsz) || !col_fits(h, tk, cr)) continue;
                const int cmin = col_min_threads(h, tk, cr);
                for (int ct : {cmin, 2 * cmin, 4 * cmin}) {
                    if (ct > col_max_threads(h, cr)) continue;
                    LaunchCfg c = cur;
                    c.tk = tk;
                    c.col_thr = ct;
                    c.col_r = cr;
                    if ((rc = apply_cfg(h, c))) break;
                    const float ms = timed([&] { return o.col(); });
                    if (rc) break;
                    if (ms < tbest) tbest = ms, best = c;
                }
                if (rc) break;
            }
            if (rc) break;
        }
    }
    // row kernels: forward (radix, threads), then backward (radix, threads, staged values)
    for (int pass = 0; pass < 2 && !rc; ++pass) {
        float tbest = 1e30f;
        const LaunchCfg base = best;
        for (int lr : {4, 8, 16}) {
            if (!radix_ok(h, lr)) continue;
            const int lmin = loc_min_threads(h, lr);
            if (lmin > 512) continue;
            std::vector<int> cand = {lmin};
            for (int lt : {128, 256, 512})
                if (lt > lmin) cand.push_back(lt);
            for (int lt : cand) {
                for (int nv : {4, 7}) {
                    if (pass == 0 && nv == 7) continue;
                    if (loc_lds_bytes(h, nv) > 163840) continue;
                    LaunchCfg c = base;
                    if (pass == 0) {
                        c.fwd_thr = lt;
                        c.fwd_r = lr;
                    } else {
                        c.bwd_thr = lt;
                        c.bwd_r = lr;
                        c.nv = nv;
                    }
                    if ((rc = apply_cfg(h, c))) break;
                    const float ms = timed([&] { return pass == 0 ? o.fwd(Lf) : o.bwd(Lb); });
                    if (rc) break;
                    if (ms < tbest) tbest = ms, best = c;
                }
                if (rc) break;
            }
            if (rc) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    return apply_cfg(h, best);
}

int check_ptr(const void* p, const char* name) {
    if (!p) return fail(LLG_EINVAL, std::string(name) + " is NULL");
    return LLG_OK;
}

// copy a caller array into / out of an instance buffer
int put(llg_handle* h, int i, int id, const void* src, size_t bytes, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(h->inst[i].tab.b[id], src, bytes, hipMemcpyDeviceToDevice, s));
    return LLG_OK;
}
int get(llg_handle* h, int i, int id, void* dst, size_t bytes, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(dst, h->inst[i].tab.b[id], bytes, hipMemcpyDeviceToDevice, s));
    return LLG_OK;
}

int create_batch(const llg_problem* probs, const llg_masks* masks, int n, llg_handle** out) {
    if (!out) return fail(LLG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!probs) return fail(LLG_EINVAL, "problem is NULL");
    if (n < 1) return fail(LLG_EINVAL, "a batch needs at least one instance");
    for (int i = 0; i < n; ++i)
        if (int rc = validate_problem(&probs[i])) return rc;
    const llg_problem& p0 = probs[0];
    for (int i = 1; i < n; ++i) {
        const llg_problem& q = probs[i];
        if (q.dtype != p0.dtype || q.terms != p0.terms || q.dt != p0.dt || q.max_steps != p0.max_steps ||
            q.ckpt_policy != p0.ckpt_policy || q.ckpt_param != p0.ckpt_param)
            return fail(LLG_EINVAL, "batch instances must share dtype, terms, dt, max_steps and checkpoint policy");
    }
    auto* h = new llg_handle();
    auto bail = [&](int code) {
        free_all(h);
        delete h;
        return code;
    };
    h->dtype = p0.dtype;
    h->tsz = p0.dtype == LLG_F64 ? 8 : 4;
    h->terms = p0.terms;
    h->demag = (p0.terms & LLG_TERM_DEMAG) != 0;
    h->policy = p0.ckpt_policy;
    h->ckpt_param = p0.ckpt_param;
    h->max_steps = p0.max_steps;
    h->K = segment_length(p0.max_steps, p0.ckpt_policy, p0.ckpt_param);
    if (p0.ckpt_policy == LLG_CKPT_BINOMIAL) {
        h->nsnap = binomial_slots(p0.max_steps, p0.ckpt_param);
    } else {
        h->nsnap = (p0.max_steps + h->K - 1) / h->K;
        if (p0.ckpt_policy == LLG_CKPT_SQRT && p0.ckpt_param == 0) h->nsnap = std::max<int64_t>(h->nsnap, h->K);
        h->halves = h->nsnap > 1 ? 2 : 1;
    }
    h->inst.resize(n);
    for (int i = 0; i < n; ++i) {
        Instance& I = h->inst[i];
        I.prob = probs[i];
        I.N = I.prob.nx * I.prob.ny * I.prob.nz;
        I.nrows = I.prob.ny * I.prob.nz;
        I.Px = padded(I.prob.nx);
        I.Py = padded(I.prob.ny);
        I.Pz = padded(I.prob.nz);
        I.Kx = I.Px / 2 + 1;
        I.ktiles = (I.Kx + spec_tile_of((int)h->tsz) - 1) / spec_tile_of((int)h->tsz);
        I.ncomp = I.prob.nz > 1 ? 6 : 4;
        I.nloc = (I.nrows + 1) / 2;
        h->max_nz = std::max(h->max_nz, I.prob.nz);
        if (I.Pz > 16) return bail(fail(LLG_ESHAPE, "nz too large"));
        // the kernels address an instance's spectrum (three components) at
        // unsigned 32-bit byte offsets from its base
        if ((size_t)3 * I.ktiles * I.nrows * spec_tile_of((int)h->tsz) * 2 * h->tsz >= ((size_t)1 << 32))
            return bail(fail(LLG_ESHAPE, "spectrum of one instance exceeds 4 GiB"));
    }
    // The packed pair of the real bins pays on wide rows (its block carries a
    // second column, which on a launch of a few dozen blocks lengthens the
    // critical path): from Px = 512 on.  The choice depends on the instance
    // alone, not on the batch or the launch tiling, so a batch computes the
    // bits of its instances' own handles and every tiling the same bits.
    for (auto& I : h->inst) I.pack = I.Kx >= 257 && I.Kx > spec_tile_of((int)h->tsz) ? 1 : 0;
    int rc;
    for (int i = 0; i < n; ++i) {
        Instance& I = h->inst[i];
        const size_t t = h->tsz, N = I.N, N3b = 3 * N * t, sm = (size_t)state_mult(h);
        // masks
        const llg_masks* mk = masks ? &masks[i] : nullptr;
        const uint8_t* src[4] = {mk ? mk->antenna : nullptr, mk ? mk->port1 : nullptr, mk ? mk->port2 : nullptr,
                                 mk ? mk->design : nullptr};
        const int ids[4] = {B_ANT, B_P1, B_P2, B_DES};
        for (int k = 0; k < 4; ++k) {
            std::vector<uint8_t> host(N, 0);
            if (src[k])
                for (size_t e = 0; e < N; ++e) {
                    if (src[k][e] > 1) return bail(fail(LLG_EINVAL, "mask values must be 0 or 1"));
                    host[e] = src[k][e];
                }
            if ((rc = alloc(h, &I.tab.b[ids[k]], N))) return bail(rc);
            if (hipMemcpy(I.tab.b[ids[k]], host.data(), N, hipMemcpyHostToDevice) != hipSuccess)
                return bail(fail(LLG_EHIP, "mask upload failed"));
            long long cnt = 0;
            for (auto v : host) cnt += v;
            if (k == 0) I.has_ant = cnt > 0;
            if (k == 1) I.n_p1 = cnt;
            if (k == 2) I.n_p2 = cnt;
            if (k == 3) I.has_design = cnt > 0;
        }
        const std::pair<int, size_t> sizes[] = {
            {B_PSI, N * t}, {B_PHI, N * t}, {B_PSIF, N * t}, {B_M, sm * N3b}, {B_ACC, N3b}, {B_YA, N3b}, {B_YB, N3b},
            {B_S, h->demag ? (size_t)3 * I.nrows * I.ktiles * spec_tile_of((int)t) * 2 * t : 0},
            {B_S2, h->demag && h->halves > 1 ? (size_t)3 * I.nrows * I.ktiles * spec_tile_of((int)t) * 2 * t : 0},
            {B_SNAP, (size_t)h->nsnap * sm * N3b}, {B_YS, (size_t)(h->K * h->halves) * 4 * N3b},
            {B_BS, (size_t)(h->K * h->halves) * 4 * N3b}, {B_ELL, N3b}, {B_U0, N3b}, {B_U1, N3b},
            {B_L0, N3b}, {B_L1, N3b}, {B_GPSI, N * 8}, {B_DJDM, N3b}, {B_DPSIE, N * 8}, {B_DPSI, N * 8},
            {B_DPHI, N * 8}, {B_PPART, (size_t)I.nloc * 2 * 8}, {B_EPART, (size_t)I.nloc * 5 * 8}, {B_SCAL, 8 * 8}};
        for (auto& sz : sizes)
            if ((rc = alloc(h, &I.tab.b[sz.first], sz.second))) return bail(rc);
        // the low part of a float state starts at zero (forward runs clear it again)
        if (hipMemset(I.tab.b[B_M], 0, sm * N3b) != hipSuccess) return bail(fail(LLG_EHIP, "state clear failed"));
        // spectrum bins past Kx inside the last x-bin tile are read by the column
        // kernel's vector loads and never written: keep them zero
        for (int id : {B_S, B_S2})
            if (I.tab.b[id] && hipMemset(I.tab.b[id], 0, (size_t)3 * I.nrows * I.ktiles * spec_tile_of((int)t) * 2 * t) != hipSuccess)
                return bail(fail(LLG_EHIP, "spectrum clear failed"));
        if (h->dtype == LLG_F32) {
            fill_params<float>(I);
            rc = upload_tables<float>(h, I);
        } else {
            fill_params<double>(I);
            rc = upload_tables<double>(h, I);
        }
        if (rc) return bail(rc);
        I.pf.ncomp = I.pd.ncomp = I.ncomp;
        h->sumN += N;
        h->sumSpec += 3.0 * I.nrows * I.Kx * 2.0 * t;
        h->sumNhat += (double)I.ncomp * (I.Pz / 2 + 1) * (I.Py / 2 + 1) * I.Kx * t;
    }
    if ((rc = choose_launch(h))) return bail(rc);
    // parameter and pointer tables
    {
        void* p;
        const size_t psz = h->dtype == LLG_F32 ? sizeof(KParams<float>) : sizeof(KParams<double>);
        if ((rc = alloc(h, &p, psz * n))) return bail(rc);
        h->ptab = p;
        std::vector<unsigned char> host(psz * n);
        for (int i = 0; i < n; ++i) {
            if (h->dtype == LLG_F32)
                std::memcpy(&host[psz * i], &h->inst[i].pf, psz);
            else
                std::memcpy(&host[psz * i], &h->inst[i].pd, psz);
        }
        if (hipMemcpy(p, host.data(), psz * n, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(LLG_EHIP, "parameter table upload failed"));
        if ((rc = alloc(h, &p, sizeof(InstTab) * n))) return bail(rc);
        h->itab = (InstTab*)p;
        std::vector<InstTab> tabs(n);
        for (int i = 0; i < n; ++i) tabs[i] = h->inst[i].tab;
        if (hipMemcpy(p, tabs.data(), sizeof(InstTab) * n, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(LLG_EHIP, "pointer table upload failed"));
        h->bf.ptab = (const KParams<float>*)h->ptab;
        h->bd.ptab = (const KParams<double>*)h->ptab;
        h->bf.itab = h->bd.itab = h->itab;
    }
    if (hipDeviceSynchronize() != hipSuccess) return bail(fail(LLG_EHIP, "device sync after create failed"));
    *out = h;
    return LLG_OK;
}

// ---- batched entry points (shared by the single-instance ABI) -------------

int b_levelset(llg_handle* h, const void* const* phi, const void* const* psi_fixed, double a, int extrude,
               void* const* psi_out, hipStream_t s) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (!phi || !psi_out) return fail(LLG_EINVAL, "pointer array is NULL");
    if (!std::isfinite(a)) return fail(LLG_EINVAL, "a must be finite");
    const int n = (int)h->inst.size();
    for (int i = 0; i < n; ++i) {
        if (int rc = check_ptr(phi[i], "phi")) return rc;
        if (int rc = check_ptr(psi_out[i], "psi_out")) return rc;
    }
    for (int i = 0; i < n; ++i) {
        const Instance& I = h->inst[i];
        const size_t np = (size_t)(extrude ? I.prob.nx * I.prob.ny : I.N) * h->tsz;
        if (int rc = put(h, i, B_PHI, phi[i], np, s)) return rc;
        if (psi_fixed && psi_fixed[i]) {
            if (int rc = put(h, i, B_PSIF, psi_fixed[i], (size_t)I.N * h->tsz, s)) return rc;
        } else {
            HIPCHK(hipMemsetAsync(I.tab.b[B_PSIF], 0, (size_t)I.N * h->tsz, s));
        }
    }
    if (h->dtype == LLG_F32)
        HIPCHK(launch_levelset<float>(h->bf, a, extrude, s));
    else
        HIPCHK(launch_levelset<double>(h->bd, a, extrude, s));
    for (int i = 0; i < n; ++i)
        if (int rc = get(h, i, B_PSI, psi_out[i], (size_t)h->inst[i].N * h->tsz, s)) return rc;
    return LLG_OK;
}

int b_levelset_vjp(llg_handle* h, const void* const* phi, const double* const* g, double a, int extrude,
                   double* const* out, hipStream_t s) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (!phi || !g || !out) return fail(LLG_EINVAL, "pointer array is NULL");
    const int n = (int)h->inst.size();
    for (int i = 0; i < n; ++i) {
        if (int rc = check_ptr(phi[i], "phi")) return rc;
        if (int rc = check_ptr(g[i], "dJdpsi")) return rc;
        if (int rc = check_ptr(out[i], "dJdphi_out")) return rc;
    }
    for (int i = 0; i < n; ++i) {
        const Instance& I = h->inst[i];
        const size_t np = (size_t)(extrude ? I.prob.nx * I.prob.ny : I.N);
        if (int rc = put(h, i, B_PHI, phi[i], np * h->tsz, s)) return rc;
        if (int rc = put(h, i, B_DPSI, g[i], (size_t)I.N * 8, s)) return rc;
    }
    if (h->dtype == LLG_F32)
        HIPCHK(launch_levelset_vjp<float>(h->bf, a, extrude, s));
    else
        HIPCHK(launch_levelset_vjp<double>(h->bd, a, extrude, s));
    for (int i = 0; i < n; ++i) {
        const Instance& I = h->inst[i];
        const size_t np = (size_t)(extrude ? I.prob.nx * I.prob.ny : I.N);
        if (int rc = get(h, i, B_DPHI, out[i], np * 8, s)) return rc;
    }
    return LLG_OK;
}

// Validation of an objective for a run of n_steps.
int check_objective(const llg_objective_spec* obj, int64_t n_steps) {
    if (!obj) return LLG_OK;
    if (obj->kind < LLG_OBJ_NONE || obj->kind > LLG_OBJ_MAG_CURVE) return fail(LLG_EINVAL, "unknown objective");
    const bool port = obj->kind == LLG_OBJ_PORT_MY2 || obj->kind == LLG_OBJ_PORT_SPECTRAL || obj->kind == LLG_OBJ_MAG_CURVE;
    if (port && (obj->n_start < 0 || obj->n_start >= n_steps)) return fail(LLG_EINVAL, "n_start must be in [0, n_steps)");
    if (obj->kind == LLG_OBJ_PORT_SPECTRAL) {
        if (obj->n_freq < 1 || obj->n_freq > 4096) return fail(LLG_EINVAL, "n_freq must be in [1, 4096]");
        if (!obj->freqs || !obj->coef) return fail(LLG_EINVAL, "spectral objective needs freqs and coef");
        for (int q = 0; q < obj->n_freq; ++q)
            if (!std::isfinite(obj->freqs[q]) || !std::isfinite(obj->coef[q]) ||
                !std::isfinite(obj->coef[obj->n_freq + q]))
                return fail(LLG_EINVAL, "freqs and coef must be finite");
    }
    if (obj->kind == LLG_OBJ_MAG_CURVE) {
        if (!obj->target || !obj->weight) return fail(LLG_EINVAL, "curve objective needs target and weight");
        for (int64_t k = 0; k < n_steps - obj->n_start; ++k)
            if (!std::isfinite(obj->target[k]) || !std::isfinite(obj->weight[k]))
                return fail(LLG_EINVAL, "target and weight must be finite");
    }
    return LLG_OK;
}

// Buffers of the spectral objective (allocated on first use, sized for
// max_steps) and the upload of its frequencies and weights.  Runs before a
// launch sequence (outside any graph capture); blocks the host.
// Per-step series buffers shared by the spectral and curve objectives.
int ensure_series(llg_handle* h, bool* tabs) {
    int rc;
    const size_t steps = (size_t)h->max_steps;
    for (auto& I : h->inst) {
        if (!I.tab.b[B_PSER]) {
            if ((rc = alloc(h, &I.tab.b[B_PSER], steps * 2 * (size_t)I.nloc * 8))) return rc;
            if ((rc = alloc(h, &I.tab.b[B_SER], steps * 2 * 8))) return rc;
            if ((rc = alloc(h, &I.tab.b[B_PSRC], steps * 2 * 8))) return rc;
            *tabs = true;
        }
    }
    return LLG_OK;
}

int upload_itab(llg_handle* h) {
    std::vector<InstTab> host(h->inst.size());
    for (size_t i = 0; i < h->inst.size(); ++i) host[i] = h->inst[i].tab;
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(h->itab, host.data(), sizeof(InstTab) * host.size(), hipMemcpyHostToDevice));
    return LLG_OK;
}

// Curve objective: series buffers and the targets and weights of the window
// steps on the device (before any launch sequence; blocks the host).
int ensure_curve(llg_handle* h, const llg_objective_spec* obj, int64_t n_steps) {
    bool tabs = false;
    int rc;
    if ((rc = ensure_series(h, &tabs))) return rc;
    if (!h->curve_tw) {
        void* p;
        if ((rc = alloc(h, &p, (size_t)h->max_steps * 2 * 8))) return rc;
        h->curve_tw = (double*)p;
    }
    if (tabs && (rc = upload_itab(h))) return rc;
    const int64_t W = n_steps - obj->n_start;
    std::vector<double> tw(2 * (size_t)W);
    for (int64_t k = 0; k < W; ++k) {
        tw[k] = obj->target[k];
        tw[W + k] = obj->weight[k];
    }
    if (tw != h->curve_host) {
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(h->curve_tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice));
        h->curve_host = tw;
    }
    return LLG_OK;
}

int ensure_spectral(llg_handle* h, const llg_objective_spec* obj) {
    const int K = obj->n_freq;
    bool tabs = false;
    int rc;
    if ((rc = ensure_series(h, &tabs))) return rc;
    if (K > h->spec_cap) {
        // captured graphs pass spec_fc by value: they must not outlive the buffer they point to
        if (!h->graphs.empty()) {
            if (h->gstream) HIPCHK(hipStreamSynchronize(h->gstream));
            drop_graphs(h);
        }
        const int cap = std::max(K, 64);
        void* p;
        if ((rc = alloc(h, &p, (size_t)cap * 3 * 8))) return rc;
        h->spec_fc = (double*)p;
        for (auto& I : h->inst)
            if ((rc = alloc(h, &I.tab.b[B_SPC], (size_t)cap * 4 * 8))) return rc;
        h->spec_cap = cap;
        h->spec_host.clear();
        tabs = true;
    }
    if (tabs && (rc = upload_itab(h))) return rc;
    std::vector<double> fc(3 * (size_t)K);
    for (int q = 0; q < K; ++q) {
        fc[q] = obj->freqs[q];
        fc[K + q] = obj->coef[q];
        fc[2 * K + q] = obj->coef[K + q];
    }
    if (fc != h->spec_host) {
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(h->spec_fc, fc.data(), fc.size() * 8, hipMemcpyHostToDevice));
        h->spec_host = fc;
    }
    h->spec_k = K;
    return LLG_OK;
}

int b_forward(llg_handle* h, const void* const* psi, const void* const* m0, double t0, int64_t n_steps,
              const llg_objective_spec* obj, void* const* m_out, double* J_dev, hipStream_t s) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (!psi || !m0) return fail(LLG_EINVAL, "pointer array is NULL");
    const int n = (int)h->inst.size();
    for (int i = 0; i < n; ++i) {
        if (int rc = check_ptr(psi[i], "psi")) return rc;
        if (int rc = check_ptr(m0[i], "m0")) return rc;
    }
    if (n_steps < 1 || n_steps > h->max_steps) return fail(LLG_EINVAL, "n_steps must be in [1, max_steps]");
    if (!std::isfinite(t0)) return fail(LLG_EINVAL, "t0 must be finite");
    if (int rc = check_objective(obj, n_steps)) return rc;
    if (obj && obj->kind == LLG_OBJ_PORT_SPECTRAL)
        if (int rc = ensure_spectral(h, obj)) return rc;
    if (obj && obj->kind == LLG_OBJ_MAG_CURVE)
        if (int rc = ensure_curve(h, obj, n_steps)) return rc;
    h->fwd_valid = false;
    for (int i = 0; i < n; ++i) {
        const size_t N = h->inst[i].N;
        if (int rc = put(h, i, B_PSI, psi[i], N * h->tsz, s)) return rc;
        if (int rc = put(h, i, B_M, m0[i], 3 * N * h->tsz, s)) return rc;
    }
    ensure_plan(h, n_steps);
    const std::vector<double> key = {0.0, (double)n_steps, t0, obj ? (double)obj->kind : -1.0,
                                     obj ? (double)obj->n_start : -1.0,
                                     obj && obj->kind == LLG_OBJ_PORT_SPECTRAL ? (double)obj->n_freq : 0.0};
    int res = 0;
    int rc = run_sequence(h, s, key, n_steps, &res, [&](hipStream_t st, int* r) {
        *r = 0;
        return h->dtype == LLG_F32 ? Ops<float>{h, st}.forward(t0, n_steps, obj)
                                   : Ops<double>{h, st}.forward(t0, n_steps, obj);
    });
    if (rc) return rc;
    record_forward(h, t0, n_steps, obj);
    for (int i = 0; i < n; ++i) {
        if (m_out && m_out[i])
            if ((rc = get(h, i, B_M, m_out[i], 3 * (size_t)h->inst[i].N * h->tsz, s))) return rc;
        if (J_dev && obj && (obj->kind == LLG_OBJ_PORT_MY2 || obj->kind == LLG_OBJ_PORT_SPECTRAL ||
                             obj->kind == LLG_OBJ_MAG_CURVE))
            if ((rc = get(h, i, B_SCAL, J_dev + i, sizeof(double), s))) return rc;
    }
    return LLG_OK;
}

int b_adjoint(llg_handle* h, const void* const* psi, const void* const* dJdm_T, const double* const* expl,
              const llg_objective_spec* obj, double* const* dJdpsi_out, void* const* dJdm0_out, hipStream_t s) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (!psi || !dJdpsi_out) return fail(LLG_EINVAL, "pointer array is NULL");
    const int n = (int)h->inst.size();
    for (int i = 0; i < n; ++i) {
        if (int rc = check_ptr(psi[i], "psi")) return rc;
        if (int rc = check_ptr(dJdpsi_out[i], "dJdpsi_out")) return rc;
    }
    if (!h->fwd_valid) return fail(LLG_ESTATE, "llg_adjoint needs a preceding llg_forward on this handle");
    if (obj && (obj->kind < LLG_OBJ_NONE || obj->kind > LLG_OBJ_MAG_CURVE)) return fail(LLG_EINVAL, "unknown objective");
    if (obj && (obj->kind == LLG_OBJ_PORT_MY2 || obj->kind == LLG_OBJ_PORT_SPECTRAL || obj->kind == LLG_OBJ_MAG_CURVE) &&
        (obj->n_start < 0 || obj->n_start >= h->n_steps))
        return fail(LLG_EINVAL, "n_start must be in [0, n_steps)");
    if (obj && (obj->kind == LLG_OBJ_PORT_SPECTRAL || obj->kind == LLG_OBJ_MAG_CURVE) &&
        (h->last_obj.kind != obj->kind || h->last_obj.n_start != obj->n_start))
        return fail(LLG_ESTATE, "the objective's sources come from the last forward: run it with the same objective");
    bool use_djdm = dJdm_T != nullptr, use_expl = expl != nullptr;
    for (int i = 0; i < n; ++i) {
        if (use_djdm && !dJdm_T[i]) use_djdm = false;
        if (use_expl && !expl[i]) use_expl = false;
    }
    for (int i = 0; i < n; ++i) {
        const size_t N = h->inst[i].N;
        if (int rc = put(h, i, B_PSI, psi[i], N * h->tsz, s)) return rc;
        if (use_djdm)
            if (int rc = put(h, i, B_DJDM, dJdm_T[i], 3 * N * h->tsz, s)) return rc;
        if (use_expl)
            if (int rc = put(h, i, B_DPSIE, expl[i], N * 8, s)) return rc;
    }
    if (int rc = prepare_adjoint(h)) return rc;
    const std::vector<double> key = {1.0, (double)h->n_steps, h->t0, obj ? (double)obj->kind : -1.0,
                                     obj ? (double)obj->n_start : -1.0, (double)use_djdm, (double)use_expl};
    int lam0 = B_L0;
    int rc0 = run_sequence(h, s, key, h->n_steps, &lam0, [&](hipStream_t st, int* r) {
        if (h->dtype == LLG_F32) {
            Ops<float> o{h, st};
            const int rc = o.adjoint(obj, use_djdm, use_expl);
            *r = o.adj_lambda0;
            return rc;
        }
        Ops<double> o{h, st};
        const int rc = o.adjoint(obj, use_djdm, use_expl);
        *r = o.adj_lambda0;
        return rc;
    });
    if (rc0) return rc0;
    for (int i = 0; i < n; ++i) {
        const size_t N = h->inst[i].N;
        if (int rc = get(h, i, B_DPSI, dJdpsi_out[i], N * 8, s)) return rc;
        if (dJdm0_out && dJdm0_out[i])
            if (int rc = get(h, i, lam0, dJdm0_out[i], 3 * N * h->tsz, s)) return rc;
    }
    return LLG_OK;
}

}  // namespace

int llg::set_error(int code, const char* msg) { return fail(code, msg); }

extern "C" {

const char* llg_last_error(void) { return g_err.c_str(); }

const char* llg_version(void) { return "llg-mi355x 0.2 (gfx950, batched)"; }

int llg_query_memory(const llg_problem* p, int64_t n_steps, int32_t policy, int32_t ckpt_param, size_t* bytes) {
    if (!p || !bytes) return fail(LLG_EINVAL, "NULL argument");
    if (n_steps < 1) return fail(LLG_EINVAL, "n_steps must be >= 1");
    if (policy != LLG_CKPT_SQRT && policy != LLG_CKPT_ALL && policy != LLG_CKPT_BINOMIAL)
        return fail(LLG_EINVAL, "unknown policy");
    if (ckpt_param < 0) return fail(LLG_EINVAL, "ckpt_param must be >= 0");
    const int64_t N3 = 3LL * p->nx * p->ny * p->nz;
    *bytes = store_bytes(N3, p->dtype == LLG_F64 ? 8 : 4, n_steps, policy, ckpt_param, p->dtype == LLG_F64 ? 1 : 2);
    return LLG_OK;
}

int llg_query_recompute(int64_t n_steps, int32_t policy, int32_t ckpt_param, int64_t* steps) {
    if (!steps) return fail(LLG_EINVAL, "NULL argument");
    if (n_steps < 1) return fail(LLG_EINVAL, "n_steps must be >= 1");
    if (policy != LLG_CKPT_SQRT && policy != LLG_CKPT_ALL && policy != LLG_CKPT_BINOMIAL)
        return fail(LLG_EINVAL, "unknown policy");
    if (ckpt_param < 0) return fail(LLG_EINVAL, "ckpt_param must be >= 0");
    *steps = recompute_steps(n_steps, policy, ckpt_param);
    return LLG_OK;
}

int llg_create(const llg_problem* p, const llg_masks* masks, llg_handle** out) { return create_batch(p, masks, 1, out); }

int llg_batch_create(const llg_problem* probs, const llg_masks* masks, int32_t n, llg_batch** out) {
    return create_batch(probs, masks, n, out);
}

int llg_destroy(llg_handle* h) {
    if (!h) return LLG_OK;
    (void)hipDeviceSynchronize();
    for (auto& r : h->prof) {
        h->ev_pool.push_back(r.a);
        h->ev_pool.push_back(r.b);
    }
    for (auto e : h->ev_pool) (void)hipEventDestroy(e);
    for (auto e : h->sync_ev) (void)hipEventDestroy(e);
    if (h->aux) (void)hipStreamDestroy(h->aux);
    drop_graphs(h);
    if (h->g_in) (void)hipEventDestroy(h->g_in);
    if (h->g_out) (void)hipEventDestroy(h->g_out);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    if (h->dp.err_host) (void)hipHostFree(h->dp.err_host);
    free_all(h);
    delete h;
    return LLG_OK;
}

int llg_batch_destroy(llg_batch* b) { return llg_destroy(b); }

int llg_batch_size(const llg_batch* b, int32_t* n) {
    if (!b || !n) return fail(LLG_EINVAL, "NULL argument");
    *n = (int32_t)b->inst.size();
    return LLG_OK;
}

int llg_launch_config(const llg_handle* h, int32_t cfg[8]) {
    if (!h || !cfg) return fail(LLG_EINVAL, "NULL argument");
    cfg[0] = h->bf.col_tk;
    cfg[1] = h->bf.col_threads;
    cfg[2] = h->bf.col_radix;
    cfg[3] = h->bf.loc_threads;
    cfg[4] = h->bf.loc_radix;
    cfg[5] = h->bf.bwd_threads;
    cfg[6] = h->bf.bwd_radix;
    cfg[7] = h->bf.loc_nv;
    return LLG_OK;
}

int llg_set_launch_config(llg_handle* h, const int32_t cfg[8]) {
    if (!h || !cfg) return fail(LLG_EINVAL, "NULL argument");
    LaunchCfg c;
    c.tk = cfg[0];
    c.col_thr = cfg[1];
    c.col_r = cfg[2];
    c.fwd_thr = cfg[3];
    c.fwd_r = cfg[4];
    c.bwd_thr = cfg[5];
    c.bwd_r = cfg[6];
    c.nv = cfg[7];
    if (int rc = check_cfg(h, c)) return rc;
    HIPCHK(hipDeviceSynchronize());
    drop_graphs(h);
    return apply_cfg(h, c);
}

int llg_autotune(llg_handle* h, hipStream_t stream) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    HIPCHK(hipDeviceSynchronize());
    drop_graphs(h);
    const bool prof = h->prof_on;
    h->prof_on = false;
    LaunchCfg best;
    const int rc = h->dtype == LLG_F32 ? autotune_typed<float>(h, stream, best) : autotune_typed<double>(h, stream, best);
    h->prof_on = prof;
    h->fwd_valid = false;
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(stream));
    return LLG_OK;
}

int llg_set_graphs(llg_handle* h, int enable) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (!enable && !h->graphs.empty()) {
        if (h->gstream) HIPCHK(hipStreamSynchronize(h->gstream));
        drop_graphs(h);
    }
    h->graphs_on = enable != 0;
    return LLG_OK;
}

int llg_profile(llg_handle* h, int enable) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (enable && counter_collection_active())
        return fail(LLG_ENOTSUP, "event-timed dispatches are not used while hardware counters are collected");
    if (int rc = drain_profile(h)) return rc;
    h->prof_on = enable > 0;
    if (enable > 0) {
        h->prof_stride = enable;
        for (auto& v : h->prof_seen) v = 0;
    }
    return LLG_OK;
}

int llg_profile_read(llg_handle* h, int32_t kind, double* ms, int64_t* launches, double* bytes, int reset) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (kind < 0 || kind >= LLG_KIND_COUNT) return fail(LLG_EINVAL, "unknown kernel kind");
    if (int rc = drain_profile(h)) return rc;
    if (ms) *ms = h->prof_ms[kind];
    if (launches) *launches = h->prof_n[kind];
    if (bytes) *bytes = h->prof_bytes[kind];
    if (reset) {
        h->prof_ms[kind] = 0;
        h->prof_n[kind] = 0;
        h->prof_bytes[kind] = 0;
    }
    return LLG_OK;
}

int llg_demag_tensor(double dx, double dy, double dz, double X, double Y, double Z, int32_t method, double* out) {
    if (!out) return fail(LLG_EINVAL, "out is NULL");
    if (!(dx > 0) || !(dy > 0) || !(dz > 0) || !std::isfinite(dx) || !std::isfinite(dy) || !std::isfinite(dz))
        return fail(LLG_EINVAL, "cell edges must be finite and > 0");
    if (!std::isfinite(X) || !std::isfinite(Y) || !std::isfinite(Z)) return fail(LLG_EINVAL, "non-finite offset");
    if (method < 0 || method > 2) return fail(LLG_EINVAL, "method must be 0, 1 or 2");
    if (method == 2 && std::sqrt(X * X + Y * Y + Z * Z) < 2.0 * std::fmax(dx, std::fmax(dy, dz)))
        return fail(LLG_EINVAL, "quadrature needs centres at least two largest cell edges apart");
    tensor_at_mode(X, Y, Z, dx, dy, dz, method, out);
    return LLG_OK;
}

int llg_fft_sizes(const llg_handle* h, int32_t* P3) {
    if (!h || !P3) return fail(LLG_EINVAL, "NULL argument");
    P3[0] = h->inst[0].Px;
    P3[1] = h->inst[0].Py;
    P3[2] = h->inst[0].Pz;
    return LLG_OK;
}

int llg_levelset_to_Ms(llg_handle* h, const void* phi, const void* psi_fixed, double a, int extrude_z, void* psi_out,
                       hipStream_t stream) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    return b_levelset(h, &phi, &psi_fixed, a, extrude_z, &psi_out, stream);
}

int llg_levelset_to_Ms_vjp(llg_handle* h, const void* phi, const double* dJdpsi, double a, int extrude_z,
                           double* dJdphi_out, hipStream_t stream) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    return b_levelset_vjp(h, &phi, &dJdpsi, a, extrude_z, &dJdphi_out, stream);
}

int llg_field(llg_handle* h, const void* psi, const void* m, double t, void* B_out, void* rhs_out, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(m, "m")) || (rc = check_ptr(B_out, "B_out"))) return rc;
    if ((rc = put(h, 0, B_PSI, psi, (size_t)h->inst[0].N * h->tsz, stream))) return rc;
    if (h->dtype == LLG_F32) return Ops<float>{h, stream}.field(m, t, B_out, rhs_out);
    return Ops<double>{h, stream}.field(m, t, B_out, rhs_out);
}

int llg_forward(llg_handle* h, const void* psi, const void* m0, double t0, int64_t n_steps, const llg_objective_spec* obj,
                void* m_out, double* J_dev, hipStream_t stream) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    return b_forward(h, &psi, &m0, t0, n_steps, obj, &m_out, J_dev, stream);
}

int llg_objective(llg_handle* h, const llg_objective_spec* obj, const void* psi, const void* m, double t, double* J_dev,
                  void* dJdm_out, double* dJdpsi_out, double* energies_dev, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    if ((rc = check_ptr(obj, "obj"))) return rc;
    if (obj->kind != LLG_OBJ_ENERGY_AREA && obj->kind != LLG_OBJ_PORT_MY2 && obj->kind != LLG_OBJ_PORT_SPECTRAL &&
        obj->kind != LLG_OBJ_MAG_CURVE)
        return fail(LLG_EINVAL, "objective kind must be ENERGY_AREA, PORT_MY2, PORT_SPECTRAL or MAG_CURVE");
    const size_t N = h->inst[0].N;
    if (obj->kind != LLG_OBJ_ENERGY_AREA) {
        if (!h->fwd_valid) return fail(LLG_ESTATE, "port objective needs a preceding llg_forward");
        if (J_dev && (rc = get(h, 0, B_SCAL, J_dev, sizeof(double), stream))) return rc;
        if (dJdm_out) HIPCHK(hipMemsetAsync(dJdm_out, 0, 3 * N * h->tsz, stream));
        if (dJdpsi_out) HIPCHK(hipMemsetAsync(dJdpsi_out, 0, N * sizeof(double), stream));
        return LLG_OK;
    }
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(m, "m"))) return rc;
    if (!(obj->E_ref > 0)) return fail(LLG_EINVAL, "E_ref must be > 0");
    if ((rc = put(h, 0, B_PSI, psi, N * h->tsz, stream))) return rc;
    if (h->dtype == LLG_F32)
        return Ops<float>{h, stream}.energy(obj, (const float*)m, t, J_dev, (float*)dJdm_out, dJdpsi_out, energies_dev);
    return Ops<double>{h, stream}.energy(obj, (const double*)m, t, J_dev, (double*)dJdm_out, dJdpsi_out, energies_dev);
}

int llg_adjoint(llg_handle* h, const void* psi, const void* dJdm_T, const double* dJdpsi_expl, const llg_objective_spec* obj,
                double* dJdpsi_out, void* dJdm0_out, hipStream_t stream) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    return b_adjoint(h, &psi, dJdm_T ? &dJdm_T : nullptr, dJdpsi_expl ? &dJdpsi_expl : nullptr, obj, &dJdpsi_out,
                     &dJdm0_out, stream);
}

int llg_batch_levelset_to_Ms(llg_batch* b, const void* const* phi, const void* const* psi_fixed, double a, int extrude_z,
                             void* const* psi_out, hipStream_t stream) {
    return b_levelset(b, phi, psi_fixed, a, extrude_z, psi_out, stream);
}

int llg_batch_levelset_to_Ms_vjp(llg_batch* b, const void* const* phi, const double* const* dJdpsi, double a,
                                 int extrude_z, double* const* dJdphi_out, hipStream_t stream) {
    return b_levelset_vjp(b, phi, dJdpsi, a, extrude_z, dJdphi_out, stream);
}

int llg_batch_forward(llg_batch* b, const void* const* psi, const void* const* m0, double t0, int64_t n_steps,
                      const llg_objective_spec* obj, void* const* m_out, double* J_dev, hipStream_t stream) {
    return b_forward(b, psi, m0, t0, n_steps, obj, m_out, J_dev, stream);
}

int llg_batch_adjoint(llg_batch* b, const void* const* psi, const void* const* dJdm_T, const double* const* dJdpsi_expl,
                      const llg_objective_spec* obj, double* const* dJdpsi_out, void* const* dJdm0_out,
                      hipStream_t stream) {
    return b_adjoint(b, psi, dJdm_T, dJdpsi_expl, obj, dJdpsi_out, dJdm0_out, stream);
}

}  // extern "C"

namespace {

// Buffers of the adaptive integrator (first use; sized for max_steps accepted steps).
int ensure_dopri(llg_handle* h) {
    auto& D = h->dp;
    if (!D.err_host) {
        void* ph = nullptr;
        if (hipHostMalloc(&ph, sizeof(double), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LLG_ENOMEM, "hipHostMalloc of the error-norm readback failed");
        }
        D.err_host = static_cast<double*>(ph);
    }
    if (D.keep && !D.stages) {
        const size_t nb = (size_t)3 * h->inst[0].N * h->tsz;
        if (int rc = alloc(h, &D.stages, nb * 11 * (size_t)(h->max_steps + 1))) return rc;
    }
    if (D.snaps) return LLG_OK;
    const size_t nb = (size_t)3 * h->inst[0].N * h->tsz;
    int rc;
    for (auto& k : D.k)
        if ((rc = alloc(h, &k, nb))) return rc;
    for (auto& m : D.mu)
        if ((rc = alloc(h, &m, nb))) return rc;
    if ((rc = alloc(h, &D.y5, nb)) || (rc = alloc(h, &D.ystage, nb)) || (rc = alloc(h, &D.ystage2, nb)) ||
        (rc = alloc(h, &D.lam, nb)))
        return rc;
    if ((rc = alloc(h, &D.snaps, nb * (size_t)(h->max_steps + 1)))) return rc;
    void* e;
    if ((rc = alloc(h, &e, (8 + (3 * h->inst[0].N + 255) / 256) * sizeof(double)))) return rc;
    D.err = (double*)e;
    return LLG_OK;
}

template <typename T>
int forward_adaptive(llg_handle* h, double t0, double t_end, double h0, double rtol, double atol, int64_t* n_rej,
                     hipStream_t s) {
    Ops<T> o{h, s};
    auto& D = h->dp;
    const size_t n3 = (size_t)3 * h->inst[0].N;
    double t = t0, hstep = h0;
    bool ok_last = true, have_k0 = false;
    int64_t rejected = 0;
    T* snaps = static_cast<T*>(D.snaps);
    while (t < t_end) {
        if ((int64_t)D.hs.size() >= h->max_steps)
            return fail(LLG_ENOMEM, "adaptive run needs more accepted steps than max_steps");
        hstep = std::min(hstep, t_end - t);
        const T* m = snaps + D.hs.size() * n3;
        if (int rc = o.dp_trial((int64_t)D.hs.size(), m, t, hstep, rtol, atol, have_k0)) return rc;
        have_k0 = true;  // a rejection keeps (m, t); an acceptance moves k[6] = f(y5, t + h) into k[0]
        HIPCHK(hipMemcpyAsync(D.err_host, D.err, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double err = *D.err_host;
        if (!std::isfinite(err)) return fail(LLG_ENONFINITE, "non-finite error estimate");
        double f = err == 0.0 ? 5.0 : std::min(5.0, std::max(0.2, 0.9 * std::pow(err, -0.2)));
        if (err <= 1.0) {
            HIPCHK(hipMemcpyAsync(snaps + (D.hs.size() + 1) * n3, D.y5, n3 * sizeof(T), hipMemcpyDeviceToDevice, s));
            D.ts.push_back(t);
            D.hs.push_back(hstep);
            t = t_end - t > hstep ? t + hstep : t_end;
            std::swap(D.k[0], D.k[6]);
            if (!ok_last) f = std::min(f, 1.0);
            hstep *= f;
            ok_last = true;
        } else {
            ++rejected;
            hstep *= std::min(f, 1.0);
            ok_last = false;
            if (!(hstep > 0.0)) return fail(LLG_ENONFINITE, "step size underflow");
        }
    }
    if (n_rej) *n_rej = rejected;
    return LLG_OK;
}

}  // namespace

extern "C" {

int llg_forward_adaptive(llg_handle* h, const void* psi, const void* m0, double t0, double t_end, double h0,
                         double rtol, double atol, void* m_out, int64_t* n_accepted, int64_t* n_rejected,
                         hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(m0, "m0"))) return rc;
    if (!std::isfinite(t0) || !std::isfinite(t_end) || !(t_end > t0)) return fail(LLG_EINVAL, "need t_end > t0");
    if (!(h0 > 0.0) || !std::isfinite(h0)) return fail(LLG_EINVAL, "h0 must be > 0");
    if (!(rtol >= 0.0) || !(atol >= 0.0) || !(rtol + atol > 0.0)) return fail(LLG_EINVAL, "need rtol, atol >= 0, not both 0");
    if (h->K * h->halves < 6) return fail(LLG_ENOTSUP, "adaptive adjoint needs 6 stage slots: raise max_steps");
    if ((rc = ensure_dopri(h))) return rc;
    auto& D = h->dp;
    D.valid = false;
    D.stages_valid = false;
    D.hs.clear();
    D.ts.clear();
    h->fwd_valid = false;
    const size_t N = h->inst[0].N;
    if ((rc = put(h, 0, B_PSI, psi, N * h->tsz, stream))) return rc;
    HIPCHK(hipMemcpyAsync(D.snaps, m0, 3 * N * h->tsz, hipMemcpyDeviceToDevice, stream));
    rc = h->dtype == LLG_F32 ? forward_adaptive<float>(h, t0, t_end, h0, rtol, atol, n_rejected, stream)
                             : forward_adaptive<double>(h, t0, t_end, h0, rtol, atol, n_rejected, stream);
    if (rc) return rc;
    if (m_out)
        HIPCHK(hipMemcpyAsync(m_out, static_cast<char*>(D.snaps) + D.hs.size() * 3 * N * h->tsz, 3 * N * h->tsz,
                              hipMemcpyDeviceToDevice, stream));
    if (n_accepted) *n_accepted = (int64_t)D.hs.size();
    D.valid = true;
    D.stages_valid = D.keep;
    return LLG_OK;
}

int llg_set_keep_stages(llg_handle* h, int keep) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    h->dp.keep = keep != 0;
    return LLG_OK;
}

int llg_adaptive_steps(const llg_handle* h, double* hs_out, int64_t cap) {
    if (!h || !hs_out) return fail(LLG_EINVAL, "NULL argument");
    if (!h->dp.valid) return fail(LLG_ESTATE, "no adaptive run recorded");
    if (cap < (int64_t)h->dp.hs.size()) return fail(LLG_EINVAL, "cap smaller than the number of accepted steps");
    std::copy(h->dp.hs.begin(), h->dp.hs.end(), hs_out);
    return LLG_OK;
}

}  // extern "C"

namespace {

int adjoint_on_kept_states(llg_handle* h, const void* psi, const void* dJdm_T, const double* dJdpsi_expl,
                           double* dJdpsi_out, void* dJdm0_out, int n_sub, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (n_sub < 0 || n_sub > 64) return fail(LLG_EINVAL, "n_sub must be in 1..64");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(dJdpsi_out, "dJdpsi_out"))) return rc;
    if (!h->dp.valid) return fail(LLG_ESTATE, "llg_adjoint_adaptive needs a preceding llg_forward_adaptive");
    const size_t N = h->inst[0].N, nb = 3 * N * h->tsz;
    if ((rc = put(h, 0, B_PSI, psi, N * h->tsz, stream))) return rc;
    if (dJdm_T)
        HIPCHK(hipMemcpyAsync(h->dp.lam, dJdm_T, nb, hipMemcpyDeviceToDevice, stream));
    else
        HIPCHK(hipMemsetAsync(h->dp.lam, 0, nb, stream));
    if (dJdpsi_expl && (rc = put(h, 0, B_DPSIE, dJdpsi_expl, N * 8, stream))) return rc;
    h->fwd_valid = false;  // the stage store now holds this run's states
    const bool ex = dJdpsi_expl != nullptr;
    if (h->dtype == LLG_F32) {
        Ops<float> o{h, stream};
        rc = n_sub ? o.continuous_adjoint(ex, n_sub) : o.dp_adjoint(ex);
    } else {
        Ops<double> o{h, stream};
        rc = n_sub ? o.continuous_adjoint(ex, n_sub) : o.dp_adjoint(ex);
    }
    if (rc) return rc;
    if ((rc = get(h, 0, B_DPSI, dJdpsi_out, N * 8, stream))) return rc;
    if (dJdm0_out) HIPCHK(hipMemcpyAsync(dJdm0_out, h->dp.lam, nb, hipMemcpyDeviceToDevice, stream));
    return LLG_OK;
}

}  // namespace

extern "C" {

int llg_adjoint_adaptive(llg_handle* h, const void* psi, const void* dJdm_T, const double* dJdpsi_expl,
                         double* dJdpsi_out, void* dJdm0_out, hipStream_t stream) {
    return adjoint_on_kept_states(h, psi, dJdm_T, dJdpsi_expl, dJdpsi_out, dJdm0_out, 0, stream);
}

int llg_adjoint_continuous(llg_handle* h, const void* psi, const void* dJdm_T, const double* dJdpsi_expl, int n_sub,
                           double* dJdpsi_out, void* dJdm0_out, hipStream_t stream) {
    if (n_sub < 1) return fail(LLG_EINVAL, "n_sub must be in 1..64");
    return adjoint_on_kept_states(h, psi, dJdm_T, dJdpsi_expl, dJdpsi_out, dJdm0_out, n_sub, stream);
}

int llg_shape_penalty(llg_handle* h, const void* psi, double xi, double S_target, double nu, double x0, double y0,
                      double* J_dev, double* dJdpsi_out, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(J_dev, "J_dev"))) return rc;
    const double vals[] = {xi, S_target, nu, x0, y0};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(LLG_EINVAL, "constraint parameters must be finite");
    const llg_problem& q = h->inst[0].prob;
    const size_t N = h->inst[0].N;
    if (!h->shape_work) {
        void* p;
        if ((rc = alloc(h, &p, (8 + 3 * ((N + 255) / 256)) * sizeof(double)))) return rc;
        h->shape_work = (double*)p;
    }
    hipError_t e = h->dtype == LLG_F32
                       ? launch_shape<float>((const float*)psi, q.nx, q.ny, q.nz, xi, S_target, nu, x0, y0,
                                             h->shape_work, J_dev, dJdpsi_out, stream)
                       : launch_shape<double>((const double*)psi, q.nx, q.ny, q.nz, xi, S_target, nu, x0, y0,
                                              h->shape_work, J_dev, dJdpsi_out, stream);
    if (e != hipSuccess) return fail(LLG_EHIP, std::string("shape constraint launch: ") + hipGetErrorString(e));
    return LLG_OK;
}

int llg_shape_penalty_noalloc(llg_handle* h, const void* psi, double xi, double S_target, double nu, double x0,
                              double y0, double* J_dev, double* dJdpsi_out, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (h->inst.size() != 1) return fail(LLG_EINVAL, "single-instance call on a batch");
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(J_dev, "J_dev"))) return rc;
    const double vals[] = {xi, S_target, nu, x0, y0};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(LLG_EINVAL, "constraint parameters must be finite");
    const llg_problem& q = h->inst[0].prob;
    const size_t N = h->inst[0].N;
    if (N > (size_t)kShapeMaxNodes)
        return fail(LLG_ENOMEM, "llg_shape_penalty_noalloc: " + std::to_string(N) + " nodes exceed its scratch (" +
                                    std::to_string(kShapeMaxNodes) + " nodes)");
    double* work = nullptr;
    hipError_t e = shape_scratch_ptr(&work);
    if (e != hipSuccess) return fail(LLG_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
    e = h->dtype == LLG_F32 ? launch_shape<float>((const float*)psi, q.nx, q.ny, q.nz, xi, S_target, nu, x0, y0, work,
                                                  J_dev, dJdpsi_out, stream)
                            : launch_shape<double>((const double*)psi, q.nx, q.ny, q.nz, xi, S_target, nu, x0, y0,
                                                   work, J_dev, dJdpsi_out, stream);
    if (e != hipSuccess) return fail(LLG_EHIP, std::string("shape constraint launch: ") + hipGetErrorString(e));
    return LLG_OK;
}

}  // extern "C"
