// Internal declarations shared by the host runtime and the device kernels.
//
// Every kernel works on a *batch* of problem instances (a single-instance
// solver is a batch of one).  Per-instance constants (KParams) and device
// buffer pointers (InstTab) sit in device tables; a work list maps each
// thread block to (instance, row pair) or (instance, column tile).  Launch
// arguments shared by all instances (stage, time, which buffer plays which
// role) travel by value, so the same launch sequence serves every instance.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

namespace llg {

constexpr double kMu0 = 4e-7 * 3.14159265358979323846;

// LDS arrays of complex values are padded by one element per 2^kLdsPadShift.
// 32 complex values fill the 64 four-byte banks once, so the pad shifts each
// such run by one element: a run of 32 contiguous points (a half wave of
// 8-byte accesses) stays on distinct banks, and strided runs rotate.
constexpr int kLdsPadShift = 5;
// Stored size of an LDS array of n padded complex values.
__host__ __device__ inline int lds_pad(int n) { return n + (n >> kLdsPadShift) + 1; }

// Spectra are stored in x-bin tiles of 128 bytes (16 float or 8 double
// complex bins): S[((c * ktiles + t) * nrows + row) * TW + o] for bin kx =
// t * TW + o, and the real tensor spectrum nhat[(t * NR + q) * TW + o] with
// q = (comp * Kz2 + kz) * Ky2 + ky, NR = ncomp * Kz2 * Ky2.  A column tile then
// reads whole 128-byte lines, and a row reads or writes one line per tile.
template <typename T> constexpr int spec_tile() { return 128 / (2 * (int)sizeof(T)); }
inline int spec_tile_of(int tsz) { return 128 / (2 * tsz); }

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };
template <typename T> using cplx = typename Cx<T>::type;

// Per-instance device buffers, addressed by role.
enum BufId : int {
    B_PSI = 0,  // material map psi (N)
    B_PHI,      // level-set input (N or nx*ny)
    B_PSIF,     // psi outside the design region (N)
    B_DES,      // design mask (u8, N)
    B_ANT,      // antenna mask (u8, N)
    B_P1,       // port-1 mask (u8, N)
    B_P2,       // port-2 mask (u8, N)
    B_M,        // magnetisation m_n (3N)
    B_ACC,      // RK accumulator (3N)
    B_YA,       // stage state (3N)
    B_YB,       // stage state (3N)
    B_S,        // x-spectrum (3 * ktiles * nrows * TW complex, tiled in x)
    B_S2,       // second x-spectrum (segment recomputation on the second stream)
    B_TWX,      // twiddles (Px), (Py), (Pz)
    B_TWY,
    B_TWZ,
    B_NHAT,     // tensor spectrum (ktiles * ncomp * Kz2 * Ky2 * TW real, tiled in x)
    B_SNAP,     // checkpoint snapshots (nsnap * 3N)
    B_YS,       // stage states of recomputed steps (slots * 4 * 3N)
    B_BS,       // fields of those stage states (slots * 4 * 3N)
    B_ELL,      // stage adjoint l_s (3N)
    B_U0,       // field adjoint u (3N), ping-pong
    B_U1,
    B_L0,       // adjoint state lambda (3N), ping-pong
    B_L1,
    B_GPSI,     // dJ/dpsi accumulator (double, N)
    B_DJDM,     // terminal dJ/dm input (3N)
    B_DPSIE,    // explicit dJ/dpsi input (double, N)
    B_DPSI,     // dJ/dpsi output (double, N)
    B_DPHI,     // dJ/dphi output (double, N or nx*ny)
    B_PPART,    // port partial sums (double, 2 per row-pair block)
    B_EPART,    // energy partial sums (double, 5 per row-pair block)
    B_SCAL,     // scalars (double[8]): [0] J, [1] area coefficient
    B_PSER,     // spectral objective: per-step port partial sums (double, max_steps * nloc * 2)
    B_SER,      // spectral objective: port-mean m_y series x_1(n), x_2(n) (double, 2 * max_steps)
    B_PSRC,     // spectral objective: per-step sources dJ/dx_j(n) / |P_j| (double, 2 * max_steps)
    B_SPC,      // spectral objective: C_1, S_1, C_2, S_2 of each sample frequency (double, 4 * capacity)
    B_COUNT
};
struct InstTab {
    void* b[B_COUNT];
};

// Per-instance constants (precision T).
template <typename T>
struct KParams {
    int nx, ny, nz, N, nrows;      // nodes; rows = ny*nz lines along x
    int Px, Kx, Py, Pz, Ky2, Kz2;  // padded FFT sizes; Kx = Px/2+1; Ky2 = Py/2+1; Kz2 = Pz/2+1
    int ktiles;                    // x-bin tiles of the stored spectra, ceil(Kx / TW)
    int pack;                      // 1: the block of bin 0 also transforms bin Px/2 (alone in the last tile)
    int ncomp;                     // stored tensor-spectrum components (4 in 2D, 6 in 3D)
    int terms;
    int nloc;                      // row-pair blocks of this instance
    int has_ant, n_p1, n_p2;       // mask populations
    T exw[3];                      // 2 kappa / h_d^2, kappa = 2 A / Ms
    T anis;                        // 2 K / Ms
    T u[3];                        // anisotropy axis
    T B0[3];
    T brf[3];
    T alpha0, alpha_max;
    int ramp_cells, ramp_faces;
    T gamma;
    T dt;
    double f1, f2, t_switch;
    int drive_kind;                // 0 sine, 1 ramp t / t_ramp
    double t_ramp;
    T psi_freeze;                  // nodes with psi <= psi_freeze are frozen (0: psi = 0 only)
};

// One forward-stage launch (shared by every instance of the batch).
struct FwdL {
    int stage;            // 0..3 RK4 stage; -1 field evaluation; -3 spectrum of psi*ys only
    double t;             // time of the stage
    int ys, mn, acc, ynext;  // BufId roles (-1 = none)
    int store_j;          // >= 0: copy ys and B(ys) to slot store_j of YS / BS
    int port;             // stage 3: 1 accumulate the port m_y^2 sums; write, for window step pstep, 2 the port
                          // m_y sums (spectral objective), 3 the psi m_x and psi sums over all nodes (curve objective)
    int pstep;            // window index of the state this launch produces (port == 2)
    int do_inv, do_fwd;   // inverse x-FFT of S (demag in) / forward x-FFT of psi*ynext into S
    int spec;             // BufId of S (B_S or B_S2)
    void* ext_ys;         // single-instance overrides (field evaluation)
    void* ext_ynext;
    void* ext_B;
    // single-instance stage sum of a field evaluation (stage -1): the launch also forms
    // Y' = lin_base + sum_j lin_c[j] lin_src[j] + lin_cf f, f the rate it computes (added last, each term one
    // fused multiply-add in this order), stores Y' at lin_out and, with do_fwd, transforms psi * Y'
    const void* lin_base;
    const void* lin_src[6];
    double lin_c[6];
    double lin_cf;
    int lin_nt;
    void* lin_out;
};

// One backward-stage launch.
struct BwdL {
    int stage;            // 3..0, or -2 seed (l = dt/6 lambda', u from y_prev)
    int j;                // slot of this step's stage states in YS / BS
    int prev_j, prev_st;  // slot and stage of y_prev (prev_j < 0: none)
    int ucur, unext, lamp, lacc;  // BufId roles
    int port_src;         // add the port running-cost source at stage 0
    int W;                // port window length (steps)
    int port_lin;         // 1 spectral, 2 curve objective: the source is the stored per-step scalar
    int pstep;            // window index of this step's state (port_lin)
    int seed_unit;        // seed stage: l = lambda' itself (a generic stage transpose) instead of dt/6 lambda'
    int do_inv, do_fwd;
    int stage_m;          // stage the y_s rows in LDS too (set by the launcher from the batch)
    // single-instance transposes on states held elsewhere (nullptr: the role buffers above): the stage state
    // (also y_prev when prev_j >= 0), its field, and the accumulator written without reading one (lacc unused)
    void* ext_ys;
    void* ext_B;
    void* ext_lacc;
    // seed stage of a single-instance transpose: l = sum_j lin_c[j] lin_src[j] (fused multiply-adds from zero,
    // in this order) instead of lambda' from lamp
    const void* lin_src[7];
    double lin_c[7];
    int lin_nt;
};

// Resolved per-instance arguments (built inside the kernels).
template <typename T>
struct StageFwdArgs {
    int stage;
    double t;
    const T* psi;
    const T* ys;
    const T* mn;
    T* acc;
    T* ynext;
    cplx<T>* S;
    const uint8_t* antenna;
    T* ys_store;
    T* Bs_store;
    const uint8_t* port1;
    const uint8_t* port2;
    double* port_part;
    int port_lin;         // 0 accumulate m_y^2; store 1 the port m_y sums, 2 the psi m_x sums over all nodes
    int do_inv;
    int do_fwd;
};

template <typename T>
struct StageBwdArgs {
    int stage;
    const T* psi;
    const T* ys;
    const T* Bs;
    const T* u_cur;
    T* ell;
    const T* lamp;
    const T* lacc_in;
    T* lacc_out;
    double* gpsi;
    const T* y_prev;
    T* u_next;
    cplx<T>* S;
    const uint8_t* port1;
    const uint8_t* port2;
    T src1, src2;         // port sources (port 2 carries its sign)
    int src_lin;          // 0 lambda.y += src m_y; 1 lambda.y += src (spectral); 2 lambda.x += src1 psi and
                          // dJ/dpsi += src1 m_x - src2 on every node (curve)
    int seed_unit;
    int do_inv;
    int do_fwd;
};

// Table pointers handed to the kernels; a batch of one passes its instance
// by value so that a block needs no dependent table loads before its work.
template <typename T>
struct BatchArgs {
    const KParams<T>* ptab;
    const InstTab* itab;
    const int2* work;
    int single;  // one instance: block b works on unit b, no work list
};

// Device-side description of a batch.
template <typename T>
struct BatchDev {
    const KParams<T>* ptab;
    const InstTab* itab;
    const int2* work_loc;  // (instance, row pair)
    const int2* work_col;  // (instance, first x-bin of the column tile), XCD-grouped
    int nloc, ncol, ninst;
    int max_n3;            // max 3N over instances (grid of element-wise kernels)
    int col_tk, col_threads, col_radix;  // column kernel: x-bins per block, block size, largest FFT radix
    int col_nt_lds;                      // column kernel stages its tensor-spectrum tile in LDS
    int loc_threads, loc_radix;          // forward row kernel (and the energy kernel's block size)
    int bwd_threads, bwd_radix;          // backward row kernel
    int loc_nv;                          // node values per staged row in the backward row kernel (4 or 7)
    int fwd_rows;                        // forward row kernel stages its neighbour rows in LDS
    size_t loc_lds, fwd_lds, bwd_lds, col_lds;  // loc_lds: rows staged (energy kernel)
};

// The three per-stage kernels take an optional event pair that the runtime
// binds to the dispatch itself (start and end of the kernel on the device).
template <typename T>
hipError_t launch_stage_fwd(const BatchDev<T>& b, const FwdL& L, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_stage_bwd(const BatchDev<T>& b, const BwdL& L, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_col_conv(const BatchDev<T>& b, int max_nz, int spec, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T>
int col_conv_vgprs(int max_nz, int radix);
template <typename T>
int stage_fwd_vgprs(int radix, int staged);
template <typename T> hipError_t launch_levelset(const BatchDev<T>& b, double a, int extrude, hipStream_t s);
template <typename T> hipError_t launch_levelset_vjp(const BatchDev<T>& b, double a, int extrude, hipStream_t s);
template <typename T>
hipError_t launch_adj_init(const BatchDev<T>& b, int lam_sel, int use_djdm, int port, int W, hipStream_t s);
template <typename T> hipError_t launch_psi_grad_out(const BatchDev<T>& b, int use_expl, hipStream_t s);
template <typename T> hipError_t launch_zero(const BatchDev<T>& b, int sel, int what, hipStream_t s);
// role[off N + e] = v for e < mult N (a fill kernel, also under graph capture)
template <typename T>
hipError_t launch_fill(const BatchDev<T>& b, int sel, int mult, double v, hipStream_t s, int off = 0);
template <typename T>
hipError_t launch_copy(const BatchDev<T>& b, int src, int src_slot, int dst, int dst_slot, int mult, hipStream_t s);
template <typename T> hipError_t launch_port_finish(const BatchDev<T>& b, int W, hipStream_t s);
// Spectral objective after a forward run: series from the per-step partials, DFT
// parts at the K sample frequencies, J, and the per-step adjoint sources.  fc
// holds f_q (K), then the weights of |X_1| (K) and of |X_2| (K), on the device.
// Curve objective after a forward run: M_x series and per-step sources, then J.
// tw holds the W targets, then the W weights, on the device.
// Linear combinations of up to 7 device vectors (explicit Runge-Kutta stages):
// out[e] = (base ? base[e] : 0) + sum_j c[j] src[j][e], e < n, in order j = 0, 1, ...
template <typename T>
struct LinTerms {
    const T* src[7];
    double c[7];
    int nt;
};
template <typename T> hipError_t launch_lincomb(int n, T* out, const T* base, const LinTerms<T>& t, hipStream_t s);
// Error norm of an embedded pair: max_e |sum_j c[j] k_j[e]| / (atol + rtol max(|y[e]|, |y5[e]|)) into *out
// (device double); part holds ceil(n / 256) doubles.
template <typename T>
hipError_t launch_err_norm(int n, const T* y, const T* y5, const LinTerms<T>& t, double rtol, double atol,
                           double* part, double* out, hipStream_t s);

// Size and centre constraints (Eq. 9) of psi (nx*ny*nz): J to J[0], dJ/dpsi to g
// (nullable); work holds 8 + 3 * ceil(N / 256) doubles.
template <typename T>
hipError_t launch_shape(const T* psi, int nx, int ny, int nz, double xi, double S_target, double nu, double x0,
                        double y0, double* work, double* J, double* g, hipStream_t s);
template <typename T> hipError_t launch_curve(const BatchDev<T>& b, const double* tw, int W, hipStream_t s);

// Allocation-free shape penalty: nodes its static scratch covers, and the
// device address of that scratch on the current device (looked up once per
// device with hipGetSymbolAddress; no allocation).
constexpr int kShapeMaxNodes = 1 << 23;
hipError_t shape_scratch_ptr(double** out);
template <typename T>
hipError_t launch_spectral(const BatchDev<T>& b, const double* fc, int K, int W, double t0, int64_t n_start, double dt,
                           hipStream_t s);
template <typename T>
hipError_t launch_energy(const BatchDev<T>& b, double t, const T* m, double scale, T* dJdm, double* dJdpsi,
                         hipStream_t s);
template <typename T>
hipError_t launch_energy_finish(const BatchDev<T>& b, double MsV, double lam, double area, double E_ref, double* J,
                                double* en, double* dJdpsi, hipStream_t s);
template <typename T> hipError_t set_lds_limits(size_t bytes);

// Records msg as the text llg_last_error() returns on this thread; returns code.
int set_error(int code, const char* msg);

// True while a profiler collects hardware counters from this process
// (rocprofv3 --pmc / counter groups export ROCPROF_COUNTER_COLLECTION).  The
// libraries' event-timed dispatches (hipExtLaunchKernelGGL with start/stop
// events) are refused then: one such run ended in a segmentation fault inside
// the HIP launch path, and counter runs need only the dispatches themselves.
inline bool counter_collection_active() {
    const char* v = getenv("ROCPROF_COUNTER_COLLECTION");
    return v && *v && strcmp(v, "0") != 0 && strcmp(v, "False") != 0 && strcmp(v, "false") != 0;
}

// Host side: tensor spectrum (float64) in the kernel layout, scaled by -mu0 Ms / (Px Py Pz).
void build_tensor_spectrum(int nx, int ny, int nz, double dx, double dy, double dz, int Px, int Py, int Pz,
                           double scale, std::vector<double>& out, int& ncomp);

// Newell tensor at one physical offset (6 components xx,yy,zz,xy,xz,yz);
// mode 0 = closed form near, quadrature far; 1 = closed form; 2 = quadrature.
void tensor_at(double X, double Y, double Z, double hx, double hy, double hz, double out[6]);
void tensor_at_mode(double X, double Y, double Z, double hx, double hy, double hz, int mode, double out[6]);

}  // namespace llg
