// Host runtime of the level-set LLG library: handle, workspace, argument
// validation, stream-ordered orchestration of the forward run, the objective,
// and the checkpointed discrete adjoint, and the extern "C" entry points.
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

}  // namespace

struct llg_handle {
    llg_problem prob{};
    int dtype = LLG_F32;
    size_t tsz = 4;  // sizeof(T)
    int N = 0, nrows = 0, Px = 1, Py = 1, Pz = 1, Kx = 1, ncomp = 4;
    bool demag = false;
    KParams<float> pf{};
    KParams<double> pd{};
    LocalLaunch loc{};
    ColLaunch col{};
    // device workspace
    std::vector<DevBuf> bufs;
    void* twx = nullptr;
    void* twy = nullptr;
    void* twz = nullptr;
    void* nhat = nullptr;
    void* S = nullptr;
    void* m = nullptr;
    void* acc = nullptr;
    void* yA = nullptr;
    void* yB = nullptr;
    uint8_t* antenna = nullptr;
    uint8_t* port1 = nullptr;
    uint8_t* port2 = nullptr;
    uint8_t* design = nullptr;
    bool has_antenna = false, has_ports = false, has_design = false;
    long long n_p1 = 0, n_p2 = 0;
    double* port_part = nullptr;
    double* en_part = nullptr;
    double* scalars = nullptr;  // [0] area coefficient
    // checkpoint store
    int64_t K = 1;        // segment length
    int64_t nsnap = 0;    // snapshot slots
    void* snaps = nullptr;
    void* YS = nullptr;   // [K][4][3N]
    void* BS = nullptr;
    // adjoint buffers
    void* L0 = nullptr;
    void* L1 = nullptr;
    void* ell = nullptr;
    void* U0 = nullptr;
    void* U1 = nullptr;
    double* gpsi = nullptr;
    // per-kernel profiling (events around every launch while enabled)
    struct ProfRec { int kind; double bytes; hipEvent_t a, b; };
    bool prof_on = false;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[LLG_KIND_COUNT] = {0};
    double prof_bytes[LLG_KIND_COUNT] = {0};
    int64_t prof_n[LLG_KIND_COUNT] = {0};
    // forward record
    bool fwd_valid = false;
    double t0 = 0.0;
    int64_t n_steps = 0;
    int64_t K_used = 1;
    llg_objective_spec last_obj{};
};

namespace {

template <typename T> KParams<T>& kp(llg_handle* h);
template <> KParams<float>& kp<float>(llg_handle* h) { return h->pf; }
template <> KParams<double>& kp<double>(llg_handle* h) { return h->pd; }

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

int64_t segment_length(int64_t n, int32_t policy, int32_t param) {
    if (n <= 0) return 1;
    if (policy == LLG_CKPT_ALL) return n;
    if (param > 0) return std::min<int64_t>(param, n);
    int64_t K = (int64_t)std::ceil(std::sqrt((double)n));
    return std::max<int64_t>(1, K);
}

size_t store_bytes(int64_t N3, size_t tsz, int64_t n, int32_t policy, int32_t param) {
    const int64_t K = segment_length(n, policy, param);
    const int64_t nsnap = (n + K - 1) / K;
    return (size_t)(nsnap * N3 + 8 * K * N3) * tsz;
}

template <typename T>
void fill_params(llg_handle* h) {
    KParams<T>& p = kp<T>(h);
    const llg_problem& q = h->prob;
    p.nx = q.nx;
    p.ny = q.ny;
    p.nz = q.nz;
    p.N = h->N;
    p.nrows = h->nrows;
    p.Px = h->Px;
    p.Kx = h->Kx;
    p.Py = h->Py;
    p.Pz = h->Pz;
    p.Ky2 = h->Py / 2 + 1;
    p.Kz2 = h->Pz / 2 + 1;
    p.ncomp = h->ncomp;
    p.terms = q.terms;
    const double kappa = 2.0 * q.A / q.Ms;
    const double hh[3] = {q.dx, q.dy, q.dz};
    for (int d = 0; d < 3; ++d) p.exw[d] = (T)(2.0 * kappa / (hh[d] * hh[d]));
    p.anis = (T)(2.0 * q.K / q.Ms);
    double un = std::sqrt(q.ku[0] * q.ku[0] + q.ku[1] * q.ku[1] + q.ku[2] * q.ku[2]);
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
}

template <typename T>
int upload_tables(llg_handle* h) {
    using C = cplx<T>;
    auto twiddles = [&](int L, void** out) -> int {
        std::vector<C> tw(L);
        for (int k = 0; k < L; ++k) {
            const double th = -2.0 * 3.14159265358979323846 * (double)k / (double)L;
            tw[k].x = (T)std::cos(th);
            tw[k].y = (T)std::sin(th);
        }
        int rc = alloc(h, out, sizeof(C) * L);
        if (rc) return rc;
        HIPCHK(hipMemcpy(*out, tw.data(), sizeof(C) * L, hipMemcpyHostToDevice));
        return LLG_OK;
    };
    int rc;
    if ((rc = twiddles(h->Px, &h->twx))) return rc;
    if ((rc = twiddles(h->Py, &h->twy))) return rc;
    if ((rc = twiddles(h->Pz, &h->twz))) return rc;
    if (h->demag) {
        const llg_problem& q = h->prob;
        std::vector<double> spec;
        int nc = 4;
        const double scale = -kMu0 * q.Ms / ((double)h->Px * h->Py * h->Pz);
        build_tensor_spectrum(q.nx, q.ny, q.nz, q.dx, q.dy, q.dz, h->Px, h->Py, h->Pz, scale, spec, nc);
        h->ncomp = nc;
        std::vector<T> st(spec.size());
        for (size_t i = 0; i < spec.size(); ++i) st[i] = (T)spec[i];
        if ((rc = alloc(h, &h->nhat, sizeof(T) * st.size()))) return rc;
        HIPCHK(hipMemcpy(h->nhat, st.data(), sizeof(T) * st.size(), hipMemcpyHostToDevice));
    }
    return LLG_OK;
}

int choose_launch(llg_handle* h) {
    const int maxreg = h->dtype == LLG_F32 ? 32 : 16;
    const size_t csz = 2 * h->tsz;
    const int nx = h->prob.nx, nz = h->prob.nz;
    // local kernels: two rows per block; LDS = three packed complex signals of
    // length Px + Px twiddles (demag) + four staged rows of four values
    {
        int thr = (3 * h->Px + maxreg - 1) / maxreg;
        thr = std::max(thr, std::min(nx, 512));
        thr = std::min(512, std::max(64, round_up(thr, 64)));
        h->loc.blocks = (h->nrows + 1) / 2;
        h->loc.threads = thr;
        h->loc.lds = (h->demag ? (size_t)4 * h->Px * csz : 0) + (size_t)16 * nx * h->tsz;
        if (3 * h->Px > maxreg * 512 || h->loc.lds > 163840)
            return fail(LLG_ESHAPE, "x extent too large for the row kernels (nx = " + std::to_string(nx) + ")");
    }
    // column kernel: TK adjacent x-bins per block, as many as keep >= 256 blocks
    {
        const int Ky2 = h->Py / 2 + 1, Kz2 = h->Pz / 2 + 1;
        auto lds_of = [&](int tk) {
            return (size_t)3 * nz * h->Py * tk * csz + (size_t)h->Py * csz + (size_t)h->ncomp * Kz2 * Ky2 * tk * h->tsz;
        };
        int tk = 8;
        while (tk > 1 && ((h->Kx + tk - 1) / tk < 256 || lds_of(tk) > 163840 || 3 * nz * h->Py * tk > maxreg * 512))
            tk /= 2;
        if (lds_of(tk) > 163840 || 3 * nz * h->Py * tk > maxreg * 512)
            return fail(LLG_ESHAPE, "y/z extent too large for the column FFT (Py = " + std::to_string(h->Py) +
                                        ", nz = " + std::to_string(nz) + ")");
        int thr = (3 * nz * h->Py * tk + maxreg - 1) / maxreg;
        thr = std::max(thr, std::min(h->Py * tk, 256));
        thr = std::min(512, std::max(64, round_up(thr, 64)));
        h->col.tk = tk;
        h->col.threads = thr;
        h->col.blocks = (h->Kx + tk - 1) / tk;
        h->col.lds = lds_of(tk);
    }
    return LLG_OK;
}

int validate_problem(const llg_problem* p) {
    if (!p) return fail(LLG_EINVAL, "problem is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LLG_EINVAL, "grid extents must be >= 1");
    if ((long long)p->nx * p->ny * p->nz > (1LL << 30)) return fail(LLG_ESHAPE, "grid too large");
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
    if (p->ckpt_policy != LLG_CKPT_SQRT && p->ckpt_policy != LLG_CKPT_ALL)
        return fail(LLG_EINVAL, "unknown checkpoint policy");
    if (p->ckpt_param < 0) return fail(LLG_EINVAL, "ckpt_param must be >= 0");
    const double* vals[] = {&p->A, &p->K, &p->f1, &p->f2, &p->t_switch};
    for (auto v : vals)
        if (!std::isfinite(*v)) return fail(LLG_EINVAL, "non-finite parameter");
    return LLG_OK;
}

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

// ---------------------------------------------------------------------------
// typed orchestration
// ---------------------------------------------------------------------------
template <typename T>
struct Ops {
    using C = cplx<T>;
    llg_handle* h;
    hipStream_t s;
    const KParams<T>& P() const { return kp<T>(h); }
    size_t N3() const { return (size_t)3 * h->N; }
    T* tp(void* p, size_t off = 0) const { return static_cast<T*>(p) + off; }

    // every kernel launch goes through here: optional event bracketing for profiling
    template <typename F>
    int run(int kind, double bytes, F&& launch) {
        hipEvent_t a = nullptr, b = nullptr;
        if (h->prof_on) {
            if (int rc = take_events(h, &a, &b)) return rc;
            HIPCHK(hipEventRecord(a, s));
        }
        hipError_t e = launch();
        if (e != hipSuccess) return fail(LLG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
        if (h->prof_on) {
            HIPCHK(hipEventRecord(b, s));
            h->prof.push_back({kind, bytes, a, b});
        }
        return LLG_OK;
    }

    // algorithmic HBM bytes of one launch (each array element read or written once)
    double spec_bytes() const { return 3.0 * h->nrows * h->Kx * 2.0 * sizeof(T); }
    double fwd_bytes(const StageFwdArgs<T>& a) const {
        const double t = sizeof(T), n = h->N;
        double b = n * 4 * t;  // ys, psi
        if (a.do_inv) b += spec_bytes();
        if (a.do_fwd) b += spec_bytes();
        switch (a.stage) {
            case 0: b += n * 6 * t; break;
            case 1: case 2: b += n * 12 * t; break;
            case 3: b += n * 6 * t; break;
            case -1: b += n * 3 * t * (a.ynext ? 2 : 1); break;
            default: break;
        }
        if (a.ys_store) b += n * 3 * t;
        if (a.Bs_store && a.stage >= 0) b += n * 3 * t;
        if (a.antenna) b += n;
        if (a.port_part) b += 2 * n;
        return b;
    }
    double bwd_bytes(const StageBwdArgs<T>& a) const {
        const double t = sizeof(T), n = h->N;
        double b = 0;
        if (a.stage < 0) {
            b = n * 13 * t + spec_bytes();
        } else {
            b = n * (16 * t + 16) + (a.stage == 3 ? 0 : n * 3 * t);
            if (a.y_prev) b += n * 9 * t;
            if (a.do_inv) b += spec_bytes();
            if (a.do_fwd) b += spec_bytes();
            if (a.port1) b += 2 * n;
        }
        return b;
    }
    double col_bytes() const {
        return 2 * spec_bytes() + (double)h->ncomp * (h->Pz / 2 + 1) * (h->Py / 2 + 1) * h->Kx * sizeof(T);
    }

    int col() {
        if (!h->demag) return LLG_OK;
        return run(LLG_KIND_COLUMN, col_bytes(), [&] {
            return launch_col_conv<T>(P(), (C*)h->S, (const T*)h->nhat, (const C*)h->twy, (const C*)h->twz, h->col, s);
        });
    }
    int fwd(const StageFwdArgs<T>& a) {
        return run(LLG_KIND_STAGE_FWD, fwd_bytes(a), [&] { return launch_stage_fwd<T>(P(), a, (const C*)h->twx, h->loc, s); });
    }
    int bwd(const StageBwdArgs<T>& a) {
        return run(LLG_KIND_STAGE_BWD, bwd_bytes(a), [&] { return launch_stage_bwd<T>(P(), a, (const C*)h->twx, h->loc, s); });
    }

    // spectrum of psi * m into S
    int prologue(const T* psi, const T* m) {
        if (!h->demag) return LLG_OK;
        StageFwdArgs<T> a{};
        a.stage = -3;
        a.psi = psi;
        a.ys = m;
        a.S = (C*)h->S;
        a.do_fwd = 1;
        return fwd(a);
    }

    // one RK4 step from h->m (spectrum of psi*m already in S); optional stage store
    int step(const T* psi, double t, bool last, T* ys_store, T* bs_store, bool port) {
        const double dt = h->prob.dt;
        const double cs[4] = {0.0, 0.5, 0.5, 1.0};
        T* y_in[4] = {tp(h->m), tp(h->yA), tp(h->yB), tp(h->yA)};
        T* y_out[4] = {tp(h->yA), tp(h->yB), tp(h->yA), tp(h->m)};
        for (int st = 0; st < 4; ++st) {
            int rc = col();
            if (rc) return rc;
            StageFwdArgs<T> a{};
            a.stage = st;
            a.t = t + cs[st] * dt;
            a.psi = psi;
            a.ys = y_in[st];
            a.mn = tp(h->m);
            a.acc = tp(h->acc);
            a.ynext = y_out[st];
            a.S = (C*)h->S;
            a.antenna = h->has_antenna ? h->antenna : nullptr;
            a.ys_store = ys_store ? ys_store + st * N3() : nullptr;
            a.Bs_store = bs_store ? bs_store + st * N3() : nullptr;
            if (st == 3 && port) {
                a.port1 = h->port1;
                a.port2 = h->port2;
                a.port_part = h->port_part;
            }
            a.do_inv = h->demag;
            a.do_fwd = h->demag && !(last && st == 3);
            if (int rc2 = fwd(a)) return rc2;
        }
        return LLG_OK;
    }

    int forward(const T* psi, const T* m0, double t0, int64_t n, const llg_objective_spec* obj, T* m_out, double* J) {
        const bool port = obj && obj->kind == LLG_OBJ_PORT_MY2;
        const int64_t K = segment_length(n, h->prob.ckpt_policy, h->prob.ckpt_param);
        const int64_t nsnap = (n + K - 1) / K;
        if (nsnap > h->nsnap || K > h->K)
            return fail(LLG_ENOMEM, "checkpoint store too small for n_steps (raise max_steps at create)");
        if (m0 != tp(h->m)) HIPCHK(hipMemcpyAsync(h->m, m0, N3() * sizeof(T), hipMemcpyDeviceToDevice, s));
        if (port) HIPCHK(launch_zero_f64(h->port_part, 2 * (size_t)h->loc.blocks, s));
        int rc = prologue(psi, tp(h->m));
        if (rc) return rc;
        for (int64_t k = 0; k < n; ++k) {
            if (k % K == 0)
                HIPCHK(hipMemcpyAsync(tp(h->snaps, (k / K) * N3()), h->m, N3() * sizeof(T), hipMemcpyDeviceToDevice, s));
            const bool in_win = port && (k + 1) > obj->n_start;
            rc = step(psi, t0 + (double)k * h->prob.dt, k == n - 1, nullptr, nullptr, in_win);
            if (rc) return rc;
        }
        if (m_out && m_out != tp(h->m))
            HIPCHK(hipMemcpyAsync(m_out, h->m, N3() * sizeof(T), hipMemcpyDeviceToDevice, s));
        if (port && J) {
            const int64_t W = n - obj->n_start;
            const double inv1 = h->n_p1 > 0 ? 1.0 / (double)h->n_p1 : 0.0;
            const double inv2 = h->n_p2 > 0 ? 1.0 / (double)h->n_p2 : 0.0;
            HIPCHK(launch_port_finish<T>(h->port_part, h->loc.blocks, inv1, inv2, W > 0 ? 1.0 / (double)W : 0.0, J, s));
        }
        h->fwd_valid = true;
        h->t0 = t0;
        h->n_steps = n;
        h->K_used = K;
        h->last_obj = obj ? *obj : llg_objective_spec{};
        return LLG_OK;
    }

    int field(const T* psi, const T* m, double t, T* B, T* rhs) {
        int rc = prologue(psi, m);
        if (rc) return rc;
        rc = col();
        if (rc) return rc;
        StageFwdArgs<T> a{};
        a.stage = -1;
        a.t = t;
        a.psi = psi;
        a.ys = m;
        a.ynext = rhs;
        a.S = (C*)h->S;
        a.antenna = h->has_antenna ? h->antenna : nullptr;
        a.Bs_store = B;
        a.do_inv = h->demag;
        a.do_fwd = 0;
        return fwd(a);
    }

    int objective(const llg_objective_spec* obj, const T* psi, const T* m, double t, double* J, T* dJdm, double* dJdpsi,
                  double* en) {
        if (obj->kind == LLG_OBJ_PORT_MY2) {
            if (!h->fwd_valid) return fail(LLG_ESTATE, "port objective needs a preceding llg_forward");
            const int64_t W = h->n_steps - obj->n_start;
            const double inv1 = h->n_p1 > 0 ? 1.0 / (double)h->n_p1 : 0.0;
            const double inv2 = h->n_p2 > 0 ? 1.0 / (double)h->n_p2 : 0.0;
            if (J) HIPCHK(launch_port_finish<T>(h->port_part, h->loc.blocks, inv1, inv2, W > 0 ? 1.0 / W : 0.0, J, s));
            if (dJdm) HIPCHK(hipMemsetAsync(dJdm, 0, N3() * sizeof(T), s));
            if (dJdpsi) HIPCHK(hipMemsetAsync(dJdpsi, 0, (size_t)h->N * sizeof(double), s));
            return LLG_OK;
        }
        int rc = prologue(psi, m);
        if (rc) return rc;
        rc = col();
        if (rc) return rc;
        const llg_problem& q = h->prob;
        const double MsV = q.Ms * q.dx * q.dy * q.dz;
        HIPCHK(launch_energy<T>(P(), t, psi, m, (const C*)h->S, (const C*)h->twx, h->has_antenna ? h->antenna : nullptr,
                                MsV / obj->E_ref, dJdm, dJdpsi, h->en_part, h->loc, s));
        HIPCHK(launch_energy_finish_raw(h->en_part, h->loc.blocks, MsV, obj->lambda, obj->area, h->N, obj->E_ref, J, en,
                                        h->scalars, dJdpsi, s));
        return LLG_OK;
    }

    int adjoint(const T* psi, const T* dJdm_T, const double* expl, const llg_objective_spec* obj, double* dJdpsi,
                T* dJdm0) {
        if (!h->fwd_valid) return fail(LLG_ESTATE, "llg_adjoint needs a preceding llg_forward on this handle");
        const int64_t n = h->n_steps, K = h->K_used;
        const double dt = h->prob.dt;
        const bool port = obj && obj->kind == LLG_OBJ_PORT_MY2 && h->has_ports;
        const int64_t nstart = port ? obj->n_start : n;
        const int64_t W = n - nstart;
        const T src1 = (T)(port && W > 0 && h->n_p1 > 0 ? 2.0 / ((double)W * h->n_p1) : 0.0);
        const T src2 = (T)(port && W > 0 && h->n_p2 > 0 ? 2.0 / ((double)W * h->n_p2) : 0.0);
        T* Lc = tp(h->L0);
        T* Lo = tp(h->L1);
        T* Uc = tp(h->U0);
        T* Uo = tp(h->U1);
        // lambda_N = dJ/dm_N (+ port source at N); h->m holds m_N
        HIPCHK(launch_adj_init<T>(P(), dJdm_T, tp(h->m), (port && W > 0) ? h->port1 : nullptr, h->port2, src1, src2, Lc, s));
        HIPCHK(launch_zero_f64(h->gpsi, (size_t)h->N, s));
        const int64_t nseg = (n + K - 1) / K;
        auto YS = [&](int64_t j, int st) { return tp(h->YS, ((size_t)j * 4 + st) * N3()); };
        auto BS = [&](int64_t j, int st) { return tp(h->BS, ((size_t)j * 4 + st) * N3()); };
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const int64_t n0 = seg * K, n1 = std::min(n, n0 + K);
            // recompute the segment, storing every stage state and field
            HIPCHK(hipMemcpyAsync(h->m, tp(h->snaps, seg * N3()), N3() * sizeof(T), hipMemcpyDeviceToDevice, s));
            int rc = prologue(psi, tp(h->m));
            if (rc) return rc;
            for (int64_t k = n0; k < n1; ++k) {
                rc = step(psi, h->t0 + (double)k * dt, k == n1 - 1, YS(k - n0, 0), BS(k - n0, 0), false);
                if (rc) return rc;
            }
            // seed: l_4 and u_4 of the segment's last step
            {
                StageBwdArgs<T> a{};
                a.stage = -2;
                a.psi = psi;
                a.lamp = Lc;
                a.ell = tp(h->ell);
                a.y_prev = YS(n1 - 1 - n0, 3);
                a.u_next = Uc;
                a.S = (C*)h->S;
                a.do_fwd = h->demag;
                if (int rc2 = bwd(a)) return rc2;
            }
            for (int64_t k = n1 - 1; k >= n0; --k) {
                const int64_t j = k - n0;
                for (int st = 3; st >= 0; --st) {
                    rc = col();
                    if (rc) return rc;
                    StageBwdArgs<T> a{};
                    a.stage = st;
                    a.psi = psi;
                    a.ys = YS(j, st);
                    a.Bs = BS(j, st);
                    a.u_cur = Uc;
                    a.ell = tp(h->ell);
                    a.lamp = Lc;
                    a.lacc_in = Lo;
                    a.lacc_out = Lo;
                    a.gpsi = h->gpsi;
                    a.y_prev = st > 0 ? YS(j, st - 1) : (k > n0 ? YS(j - 1, 3) : nullptr);
                    a.u_next = Uo;
                    a.S = (C*)h->S;
                    if (st == 0 && port && k > nstart) {
                        a.port1 = h->port1;
                        a.port2 = h->port2;
                        a.src1 = src1;
                        a.src2 = src2;
                    }
                    a.do_inv = h->demag;
                    a.do_fwd = h->demag && a.y_prev != nullptr;
                    if (int rc2 = bwd(a)) return rc2;
                    if (a.y_prev) std::swap(Uc, Uo);
                }
                std::swap(Lc, Lo);  // lambda_k is the lambda' of step k-1
            }
        }
        HIPCHK(launch_psi_grad_out<T>(P(), h->gpsi, expl, dJdpsi, s));
        if (dJdm0) HIPCHK(hipMemcpyAsync(dJdm0, Lc, N3() * sizeof(T), hipMemcpyDeviceToDevice, s));
        return LLG_OK;
    }
};

int check_ptr(const void* p, const char* name) {
    if (!p) return fail(LLG_EINVAL, std::string(name) + " is NULL");
    return LLG_OK;
}

}  // namespace

extern "C" {

const char* llg_last_error(void) { return g_err.c_str(); }

const char* llg_version(void) { return "llg-mi355x 0.1 (gfx950)"; }

int llg_query_memory(const llg_problem* p, int64_t n_steps, int32_t policy, int32_t ckpt_param, size_t* bytes) {
    if (!p || !bytes) return fail(LLG_EINVAL, "NULL argument");
    if (n_steps < 1) return fail(LLG_EINVAL, "n_steps must be >= 1");
    if (policy != LLG_CKPT_SQRT && policy != LLG_CKPT_ALL) return fail(LLG_EINVAL, "unknown policy");
    const int64_t N3 = 3LL * p->nx * p->ny * p->nz;
    *bytes = store_bytes(N3, p->dtype == LLG_F64 ? 8 : 4, n_steps, policy, ckpt_param);
    return LLG_OK;
}

int llg_create(const llg_problem* p, const llg_masks* masks, llg_handle** out) {
    if (!out) return fail(LLG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_problem(p);
    if (rc) return rc;
    auto* h = new llg_handle();
    h->prob = *p;
    h->dtype = p->dtype;
    h->tsz = p->dtype == LLG_F64 ? 8 : 4;
    h->N = p->nx * p->ny * p->nz;
    h->nrows = p->ny * p->nz;
    h->Px = padded(p->nx);
    h->Py = padded(p->ny);
    h->Pz = padded(p->nz);
    h->Kx = h->Px / 2 + 1;
    h->demag = (p->terms & LLG_TERM_DEMAG) != 0;
    h->ncomp = p->nz > 1 ? 6 : 4;
    auto bail = [&](int code) {
        free_all(h);
        delete h;
        return code;
    };
    if (h->Pz > 16) return bail(fail(LLG_ESHAPE, "nz too large"));
    if ((rc = choose_launch(h))) return bail(rc);
    {
        // kernels may use more than the default 64 KiB of dynamic LDS only after opting in
        const size_t need = std::max(h->loc.lds, h->col.lds);
        if (need > 65536) {
            hipError_t e = set_lds_limits((int)need);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return bail(fail(LLG_ESHAPE, "kernel needs " + std::to_string(need) +
                                                 " bytes of LDS: " + hipGetErrorString(e)));
            }
        }
    }
    if (h->dtype == LLG_F32) {
        fill_params<float>(h);
        rc = upload_tables<float>(h);
    } else {
        fill_params<double>(h);
        rc = upload_tables<double>(h);
    }
    if (rc) return bail(rc);
    h->pf.ncomp = h->ncomp;
    h->pd.ncomp = h->ncomp;
    const size_t N3b = (size_t)3 * h->N * h->tsz;
    const size_t Sb = (size_t)3 * h->nrows * h->Kx * 2 * h->tsz;
    void** vecs[] = {&h->m, &h->acc, &h->yA, &h->yB, &h->L0, &h->L1, &h->ell, &h->U0, &h->U1};
    for (auto v : vecs)
        if ((rc = alloc(h, v, N3b))) return bail(rc);
    if (h->demag && (rc = alloc(h, &h->S, Sb))) return bail(rc);
    void* tmp;
    if ((rc = alloc(h, &tmp, (size_t)h->N * sizeof(double)))) return bail(rc);
    h->gpsi = (double*)tmp;
    if ((rc = alloc(h, &tmp, (size_t)h->loc.blocks * 2 * sizeof(double)))) return bail(rc);
    h->port_part = (double*)tmp;
    if ((rc = alloc(h, &tmp, (size_t)h->loc.blocks * 5 * sizeof(double)))) return bail(rc);
    h->en_part = (double*)tmp;
    if ((rc = alloc(h, &tmp, 8 * sizeof(double)))) return bail(rc);
    h->scalars = (double*)tmp;
    // masks
    const uint8_t* src[4] = {masks ? masks->antenna : nullptr, masks ? masks->port1 : nullptr,
                             masks ? masks->port2 : nullptr, masks ? masks->design : nullptr};
    uint8_t** dst[4] = {&h->antenna, &h->port1, &h->port2, &h->design};
    for (int k = 0; k < 4; ++k) {
        if ((rc = alloc(h, &tmp, (size_t)h->N))) return bail(rc);
        *dst[k] = (uint8_t*)tmp;
        std::vector<uint8_t> host((size_t)h->N, 0);
        if (src[k]) {
            for (int i = 0; i < h->N; ++i) {
                if (src[k][i] > 1) return bail(fail(LLG_EINVAL, "mask values must be 0 or 1"));
                host[i] = src[k][i];
            }
        }
        if (hipMemcpy(tmp, host.data(), (size_t)h->N, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(LLG_EHIP, "mask upload failed"));
        long long cnt = 0;
        for (auto v : host) cnt += v;
        if (k == 0) h->has_antenna = cnt > 0;
        if (k == 1) h->n_p1 = cnt;
        if (k == 2) h->n_p2 = cnt;
        if (k == 3) h->has_design = cnt > 0;
    }
    h->has_ports = (h->n_p1 + h->n_p2) > 0;
    // checkpoint store sized for max_steps
    h->K = segment_length(p->max_steps, p->ckpt_policy, p->ckpt_param);
    h->nsnap = (p->max_steps + h->K - 1) / h->K;
    // a shorter run under the SQRT policy uses a shorter K but more segments are never needed than for max_steps
    if (p->ckpt_policy == LLG_CKPT_SQRT && p->ckpt_param == 0) h->nsnap = std::max<int64_t>(h->nsnap, h->K);
    if ((rc = alloc(h, &h->snaps, (size_t)h->nsnap * N3b))) return bail(rc);
    if ((rc = alloc(h, &h->YS, (size_t)h->K * 4 * N3b))) return bail(rc);
    if ((rc = alloc(h, &h->BS, (size_t)h->K * 4 * N3b))) return bail(rc);
    if (hipDeviceSynchronize() != hipSuccess) return bail(fail(LLG_EHIP, "device sync after create failed"));
    *out = h;
    return LLG_OK;
}

int llg_destroy(llg_handle* h) {
    if (!h) return LLG_OK;
    (void)hipDeviceSynchronize();
    for (auto& r : h->prof) {
        h->ev_pool.push_back(r.a);
        h->ev_pool.push_back(r.b);
    }
    for (auto e : h->ev_pool) (void)hipEventDestroy(e);
    free_all(h);
    delete h;
    return LLG_OK;
}

int llg_profile(llg_handle* h, int enable) {
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if (int rc = drain_profile(h)) return rc;
    h->prof_on = enable != 0;
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

int llg_fft_sizes(const llg_handle* h, int32_t* P3) {
    if (!h || !P3) return fail(LLG_EINVAL, "NULL argument");
    P3[0] = h->Px;
    P3[1] = h->Py;
    P3[2] = h->Pz;
    return LLG_OK;
}

int llg_levelset_to_Ms(llg_handle* h, const void* phi, const void* psi_fixed, double a, int extrude_z, void* psi_out,
                       hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if ((rc = check_ptr(phi, "phi")) || (rc = check_ptr(psi_out, "psi_out"))) return rc;
    if (!std::isfinite(a)) return fail(LLG_EINVAL, "a must be finite");
    if (h->dtype == LLG_F32)
        HIPCHK(launch_levelset<float>(h->pf, (const float*)phi, (const float*)psi_fixed, h->design, a, extrude_z,
                                      (float*)psi_out, stream));
    else
        HIPCHK(launch_levelset<double>(h->pd, (const double*)phi, (const double*)psi_fixed, h->design, a, extrude_z,
                                       (double*)psi_out, stream));
    return LLG_OK;
}

int llg_levelset_to_Ms_vjp(llg_handle* h, const void* phi, const double* dJdpsi, double a, int extrude_z,
                           double* dJdphi_out, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if ((rc = check_ptr(phi, "phi")) || (rc = check_ptr(dJdpsi, "dJdpsi")) || (rc = check_ptr(dJdphi_out, "dJdphi_out")))
        return rc;
    if (h->dtype == LLG_F32)
        HIPCHK(launch_levelset_vjp<float>(h->pf, (const float*)phi, dJdpsi, h->design, a, extrude_z, dJdphi_out, stream));
    else
        HIPCHK(launch_levelset_vjp<double>(h->pd, (const double*)phi, dJdpsi, h->design, a, extrude_z, dJdphi_out, stream));
    return LLG_OK;
}

int llg_field(llg_handle* h, const void* psi, const void* m, double t, void* B_out, void* rhs_out, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(m, "m")) || (rc = check_ptr(B_out, "B_out"))) return rc;
    if (h->dtype == LLG_F32)
        return Ops<float>{h, stream}.field((const float*)psi, (const float*)m, t, (float*)B_out, (float*)rhs_out);
    return Ops<double>{h, stream}.field((const double*)psi, (const double*)m, t, (double*)B_out, (double*)rhs_out);
}

int llg_forward(llg_handle* h, const void* psi, const void* m0, double t0, int64_t n_steps, const llg_objective_spec* obj,
                void* m_out, double* J_dev, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(m0, "m0"))) return rc;
    if (n_steps < 1 || n_steps > h->prob.max_steps)
        return fail(LLG_EINVAL, "n_steps must be in [1, max_steps]");
    if (!std::isfinite(t0)) return fail(LLG_EINVAL, "t0 must be finite");
    if (obj && (obj->kind < LLG_OBJ_NONE || obj->kind > LLG_OBJ_PORT_MY2)) return fail(LLG_EINVAL, "unknown objective");
    if (obj && obj->kind == LLG_OBJ_PORT_MY2 && (obj->n_start < 0 || obj->n_start >= n_steps))
        return fail(LLG_EINVAL, "n_start must be in [0, n_steps)");
    h->fwd_valid = false;
    if (h->dtype == LLG_F32)
        return Ops<float>{h, stream}.forward((const float*)psi, (const float*)m0, t0, n_steps, obj, (float*)m_out, J_dev);
    return Ops<double>{h, stream}.forward((const double*)psi, (const double*)m0, t0, n_steps, obj, (double*)m_out, J_dev);
}

int llg_objective(llg_handle* h, const llg_objective_spec* obj, const void* psi, const void* m, double t, double* J_dev,
                  void* dJdm_out, double* dJdpsi_out, double* energies_dev, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if ((rc = check_ptr(obj, "obj"))) return rc;
    if (obj->kind != LLG_OBJ_ENERGY_AREA && obj->kind != LLG_OBJ_PORT_MY2)
        return fail(LLG_EINVAL, "objective kind must be ENERGY_AREA or PORT_MY2");
    if (obj->kind == LLG_OBJ_ENERGY_AREA) {
        if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(m, "m"))) return rc;
        if (!(obj->E_ref > 0)) return fail(LLG_EINVAL, "E_ref must be > 0");
    }
    if (h->dtype == LLG_F32)
        return Ops<float>{h, stream}.objective(obj, (const float*)psi, (const float*)m, t, J_dev, (float*)dJdm_out,
                                               dJdpsi_out, energies_dev);
    return Ops<double>{h, stream}.objective(obj, (const double*)psi, (const double*)m, t, J_dev, (double*)dJdm_out,
                                            dJdpsi_out, energies_dev);
}

int llg_adjoint(llg_handle* h, const void* psi, const void* dJdm_T, const double* dJdpsi_expl, const llg_objective_spec* obj,
                double* dJdpsi_out, void* dJdm0_out, hipStream_t stream) {
    int rc;
    if (!h) return fail(LLG_EINVAL, "handle is NULL");
    if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(dJdpsi_out, "dJdpsi_out"))) return rc;
    if (h->dtype == LLG_F32)
        return Ops<float>{h, stream}.adjoint((const float*)psi, (const float*)dJdm_T, dJdpsi_expl, obj, dJdpsi_out,
                                             (float*)dJdm0_out);
    return Ops<double>{h, stream}.adjoint((const double*)psi, (const double*)dJdm_T, dJdpsi_expl, obj, dJdpsi_out,
                                          (double*)dJdm0_out);
}

}  // extern "C"
