// Internal declarations shared by the host runtime and the device kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

namespace llg {

constexpr double kMu0 = 4e-7 * 3.14159265358979323846;

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };
template <typename T> using cplx = typename Cx<T>::type;

// Per-problem constants handed to every kernel by value (precision T).
template <typename T>
struct KParams {
    int nx, ny, nz, N, nrows;      // nodes; rows = ny*nz lines along x
    int Px, Kx, Py, Pz, Ky2, Kz2;  // padded FFT sizes; Kx = Px/2+1; Ky2 = Py/2+1; Kz2 = Pz/2+1
    int ncomp;                     // stored tensor-spectrum components (4 in 2D, 6 in 3D)
    int terms;
    T exw[3];          // 2 kappa / h_d^2, kappa = 2 A / Ms
    T anis;            // 2 K / Ms
    T u[3];            // anisotropy axis
    T B0[3];
    T brf[3];
    T alpha0, alpha_max;
    int ramp_cells, ramp_faces;
    T gamma;
    T dt;
    double f1, f2, t_switch;
};

// Launch geometry chosen on the host.
struct LocalLaunch { int blocks, threads; size_t lds; };
struct ColLaunch { int blocks, threads, tk; size_t lds; };

// Buffers of one RK stage (forward) evaluation.
template <typename T>
struct StageFwdArgs {
    int stage;             // 0..3 (RK4 stage); -1: field evaluation; -3: spectrum of psi*ys only
    double t;              // time of the stage
    const T* psi;
    const T* ys;           // stage input state (3N)
    const T* mn;           // state at the start of the step (stages 1, 2)
    T* acc;                // RK accumulator
    T* ynext;              // next stage input / m_{n+1} at stage 3 / rhs output for stage -1
    cplx<T>* S;            // x-spectrum rows (in place)
    const uint8_t* antenna;
    T* ys_store;           // optional copy of ys (adjoint recompute)
    T* Bs_store;           // optional copy of B(ys) (adjoint recompute / field output)
    const uint8_t* port1;  // optional port running cost (stage 3)
    const uint8_t* port2;
    double* port_part;     // per-block partial sums (2 per block)
    int do_inv;            // inverse x-FFT of S gives the demag field
    int do_fwd;            // forward x-FFT of psi*ynext into S
};

template <typename T>
struct StageBwdArgs {
    int stage;             // 3..0, or -2: seed only (l = dt/6 lambda', u from y_prev)
    const T* psi;
    const T* ys;           // stage state y_s
    const T* Bs;           // field at y_s
    const T* u_cur;        // u_s at every node
    T* ell;                // in: l_s, out: l_{s-1} (or l_4 of the previous step)
    const T* lamp;         // lambda' of the step
    const T* lacc_in;      // running lambda sum (stage 3 reads lamp instead)
    T* lacc_out;
    double* gpsi;          // dJ/dpsi accumulator
    const T* y_prev;       // y_{s-1}, or y_4 of step n-1 at stage 0; NULL = no chaining
    T* u_next;
    cplx<T>* S;            // conv(u_s) spectrum in, spectrum of u_next out
    const uint8_t* port1;  // port source at stage 0 (NULL = none)
    const uint8_t* port2;
    T src1, src2;          // 2/(|W| |P1|), 2/(|W| |P2|)
    int do_inv;
    int do_fwd;
};

template <typename T>
hipError_t launch_stage_fwd(const KParams<T>& p, const StageFwdArgs<T>& a, const cplx<T>* twx,
                            const LocalLaunch& L, hipStream_t s);
template <typename T>
hipError_t launch_stage_bwd(const KParams<T>& p, const StageBwdArgs<T>& a, const cplx<T>* twx,
                            const LocalLaunch& L, hipStream_t s);
template <typename T>
hipError_t launch_col_conv(const KParams<T>& p, cplx<T>* S, const T* nhat, const cplx<T>* twy,
                           const cplx<T>* twz, const ColLaunch& L, hipStream_t s);
template <typename T>
hipError_t launch_levelset(const KParams<T>& p, const T* phi, const T* psi_fixed, const uint8_t* design, double a,
                           int extrude, T* psi_out, hipStream_t s);
template <typename T>
hipError_t launch_levelset_vjp(const KParams<T>& p, const T* phi, const double* g, const uint8_t* design, double a,
                               int extrude, double* out, hipStream_t s);
template <typename T>
hipError_t launch_energy(const KParams<T>& p, double t, const T* psi, const T* m, const cplx<T>* S,
                         const cplx<T>* twx, const uint8_t* antenna, double scale, T* dJdm, double* dJdpsi,
                         double* part, const LocalLaunch& L, hipStream_t s);
hipError_t launch_energy_finish_raw(const double* part, int nb, double MsV, double lam, double area, int N,
                                    double E_ref, double* J, double* en, double* coef, double* dJdpsi,
                                    hipStream_t s);
hipError_t set_lds_limits(int bytes);
template <typename T>
hipError_t launch_port_finish(const double* part, int nblocks, double inv1, double inv2, double invW, double* J,
                              hipStream_t s);
template <typename T>
hipError_t launch_adj_init(const KParams<T>& p, const T* dJdm_T, const T* mN, const uint8_t* port1,
                           const uint8_t* port2, T src1, T src2, T* lam, hipStream_t s);
template <typename T>
hipError_t launch_psi_grad_out(const KParams<T>& p, const double* gacc, const double* expl, double* out,
                               hipStream_t s);
hipError_t launch_zero_f64(double* p, size_t n, hipStream_t s);

// Host side: tensor spectrum (float64) in the kernel layout, scaled by -mu0 Ms / (Px Py Pz).
void build_tensor_spectrum(int nx, int ny, int nz, double dx, double dy, double dz, int Px, int Py, int Pz,
                           double scale, std::vector<double>& out, int& ncomp);

// Newell tensor at one physical offset (6 components xx,yy,zz,xy,xz,yz).
void tensor_at(double X, double Y, double Z, double hx, double hy, double hz, double out[6]);

}  // namespace llg
