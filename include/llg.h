/*
 * llg.h -- C ABI of the MI355X (gfx950) level-set LLG forward/adjoint library.
 *
 * The library integrates the Landau-Lifshitz-Gilbert equation (paper: Methods,
 * Eq. 11) on a nodal finite-difference grid whose material maps follow a
 * level-set function through a smoothed Heaviside (Eq. 4 and the paragraph
 * after it), evaluates an objective of the trajectory, and returns the
 * gradient of that objective with respect to the material map by an adjoint
 * integration backwards in time (Eqs. 6-7; here the exact discrete adjoint of
 * the fixed-step RK4 map, with checkpointing so memory grows like
 * sqrt(n_steps) rather than n_steps).
 *
 * Conventions shared by every entry point
 *   - Return value: LLG_OK (0) or a negative LLG_E* code.  llg_last_error()
 *     returns a message for the calling thread's last failure.  Arguments are
 *     validated on the host before any device work is enqueued; on error no
 *     work is enqueued and no output is modified.
 *   - Arrays are caller-owned DEVICE pointers unless stated otherwise.  The
 *     library never frees them and keeps no reference after the call returns.
 *     It owns only the workspace inside an llg_handle.
 *   - Floating-point arrays are in the handle's precision (LLG_F32 -> float,
 *     LLG_F64 -> double) unless the parameter is declared double*.
 *   - Layout: node (ix, iy, iz) has flat index ix + nx*(iy + ny*iz) (x fastest).
 *     Vector fields are component-major: component c of node i at
 *     c*N + i, N = nx*ny*nz.
 *   - Work is enqueued asynchronously on the given hipStream_t (0 = the null
 *     stream); scalar results go to device memory, so no call blocks the host
 *     except llg_create/llg_destroy.
 *   - SI units: m, s, A/m, J/m, J/m^3, T, Hz.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef LLG_H
#define LLG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LLG_OK 0
#define LLG_EINVAL (-1)     /* invalid argument (null pointer, bad value)          */
#define LLG_ESHAPE (-2)     /* unsupported or inconsistent grid / FFT size         */
#define LLG_ENOMEM (-3)     /* device allocation failed or capacity exceeded       */
#define LLG_EHIP (-4)       /* a HIP runtime call failed                           */
#define LLG_ENONFINITE (-5) /* non-finite value found where one is checked         */
#define LLG_ENOTSUP (-6)    /* feature not supported for this configuration        */
#define LLG_ESTATE (-7)     /* call order violated (e.g. adjoint without forward)  */

/* ---- enums ----------------------------------------------------------- */
#define LLG_F32 0
#define LLG_F64 1

/* effective-field terms (bitmask) */
#define LLG_TERM_EXCH 1   /* exchange: kappa sum_j c_ij (m_j - m_i), harmonic-mean psi weights */
#define LLG_TERM_DEMAG 2  /* dipole-dipole field by zero-padded FFT convolution with the Newell tensor */
#define LLG_TERM_ZEEMAN 4 /* uniform bias B0 plus the drive on the antenna mask */
#define LLG_TERM_ANIS 8   /* uniaxial anisotropy (2 K / Ms)(m.u) u */

/* faces carrying the absorbing damping ramp (bitmask) */
#define LLG_FACE_XLO 1
#define LLG_FACE_XHI 2
#define LLG_FACE_YLO 4
#define LLG_FACE_YHI 8
#define LLG_FACE_ZLO 16
#define LLG_FACE_ZHI 32

/* checkpoint policies of the adjoint */
#define LLG_CKPT_SQRT 0     /* snapshots every K steps (K = ckpt_param or ceil(sqrt(n))), segments recomputed;
                               with more than one segment the stage store is double-buffered so the next
                               segment is recomputed on a second stream while the current one is transposed */
#define LLG_CKPT_ALL 1      /* one segment: every stage state of the run is kept (memory ~ n_steps) */
#define LLG_CKPT_BINOMIAL 2 /* ckpt_param snapshot slots (0 = 32) and the stage store of one step; binomial
                               (Revolve-type) recomputation schedule: memory independent of n_steps, each
                               step recomputed at most r times with C(s + r, s) >= n_steps */

/* objectives */
#define LLG_OBJ_NONE 0
#define LLG_OBJ_ENERGY_AREA 1 /* J = (E_ex + E_d)(m_T)/E_ref + lambda (mean psi - area)^2            */
#define LLG_OBJ_PORT_MY2 2    /* J = 1/|W| sum_{n in W} [mean_P1 m_y^2 - mean_P2 m_y^2], W = (n_start, n_steps] */
/* Eq. 10: J = sum_q coef[q] |X_1(f_q)| + coef[n_freq + q] |X_2(f_q)|, with X_j(f) = 1/|W| sum_{n in W}
 * x_j(n) exp(-2 pi i f t_n), x_j(n) the mean m_y over port j of the state m_n at t_n = t0 + n dt
 * (frequency windows around f1 and f2 are sets of sample frequencies f_q with coefficients +-1) */
#define LLG_OBJ_PORT_SPECTRAL 3
/* Eq. 8: J = sum_{n in W} weight[n'] |M_x(n) - target[n']|, n' = n - n_start - 1, with
 * M_x(n) = sum_i psi_i m_x,i(n) / sum_i psi_i the particle's average x component in units of Ms
 * (0 without material; explicit in psi as well as in m).  The Stoner-Wohlfarth section's
 * target M = 2 H_ext along the ramp 0 -> 0.3 Ms is target[n'] = 0.6 n / n_steps with
 * weight[n'] = 1 / (target[n'] n_steps). */
#define LLG_OBJ_MAG_CURVE 4

/* ---- problem description --------------------------------------------- */
typedef struct llg_problem {
    int32_t nx, ny, nz;       /* nodes per axis, each >= 1                                  */
    double dx, dy, dz;        /* node spacing = control-volume edges, m                     */
    double Ms;                /* saturation magnetisation of the full material, A/m (> 0)    */
    double A;                 /* exchange stiffness, J/m                                    */
    double K;                 /* uniaxial anisotropy constant, J/m^3                         */
    double ku[3];             /* anisotropy axis (normalised by the library)                */
    double gamma;             /* gyromagnetic ratio, rad/(s T)                              */
    double alpha0;            /* Gilbert damping in the bulk                                */
    double alpha_max;         /* damping on a ramped face                                   */
    int32_t ramp_cells;       /* ramp width W in nodes: alpha0 + (alpha_max-alpha0) max(0,(W-d)/W) */
    int32_t ramp_faces;       /* LLG_FACE_* bitmask                                         */
    double B0[3];             /* uniform bias field, T                                      */
    double b_rf[3];           /* drive amplitude, T: b_rf sin(phase(t)) on the antenna mask */
    double f1, f2, t_switch;  /* drive frequency f1, switching to f2 at t_switch (> 0) with a continuous phase */
    int32_t terms;            /* LLG_TERM_* bitmask                                         */
    int32_t dtype;            /* LLG_F32 or LLG_F64                                         */
    double dt;                /* RK4 step, s (> 0)                                          */
    int64_t max_steps;        /* largest n_steps a later llg_forward may use (sizes snapshots) */
    int32_t ckpt_policy;      /* LLG_CKPT_*                                                 */
    int32_t ckpt_param;       /* SQRT: segment length K (0 = ceil(sqrt(n_steps)));
                                 BINOMIAL: snapshot slots (0 = 32)                            */
    int32_t drive_kind;       /* LLG_DRIVE_*                                                */
    double t_ramp;            /* LLG_DRIVE_RAMP: time at which the drive reaches b_rf, s (> 0) */
    double psi_freeze;        /* nodes with psi <= psi_freeze carry no dynamics (dm/dt = 0); their psi
                                 still weights the exchange and the demag source.  0 (the method as
                                 stated): only psi = 0 is frozen.  An option beyond the paper: a small
                                 threshold (1e-3) keeps long driven runs' gradients reproducible, which
                                 the nearly massless interface nodes of a smoothed level set otherwise
                                 make chaotic.  0 <= psi_freeze < 1. */
} llg_problem;

/* Drive waveforms on the antenna mask */
#define LLG_DRIVE_SINE 0 /* b_rf sin(2 pi f1 t); f2 at t_switch > 0; with f2 > 0 and no switch both tones summed */
#define LLG_DRIVE_RAMP 1 /* b_rf t / t_ramp: the linear field ramp of a magnetisation curve (Eq. 8) */

/* Host-side copies of the u8 masks (length N, values 0/1); NULL = all zero.
 * They are copied into the handle by llg_create. */
typedef struct llg_masks {
    const uint8_t* antenna; /* nodes that receive the drive field            */
    const uint8_t* port1;   /* output window 1 of the port objective          */
    const uint8_t* port2;   /* output window 2 of the port objective          */
    const uint8_t* design;  /* nodes whose psi follows the level set          */
} llg_masks;

typedef struct llg_objective_spec {
    int32_t kind;     /* LLG_OBJ_*                                                   */
    double E_ref;     /* energy normalisation of LLG_OBJ_ENERGY_AREA, J (> 0)        */
    double lambda;    /* weight of the area penalty                                  */
    double area;      /* target mean psi of the area penalty                         */
    int64_t n_start;  /* port objectives: steps n with n_start < n <= n_steps count  */
    int32_t n_freq;   /* LLG_OBJ_PORT_SPECTRAL: number of sample frequencies (1..4096) */
    const double* freqs;  /* host, n_freq sample frequencies f_q, Hz                */
    const double* coef;   /* host, 2 n_freq weights: of |X_1(f_q)|, then of |X_2(f_q)| */
    const double* target; /* LLG_OBJ_MAG_CURVE: host, n_steps - n_start target values   */
    const double* weight; /* LLG_OBJ_MAG_CURVE: host, n_steps - n_start weights          */
} llg_objective_spec;

typedef struct llg_handle llg_handle;
/* A batch of instances integrated together: every kernel launch of a batch
 * call serves all of its instances (one launch per stage for the whole batch). */
typedef struct llg_handle llg_batch;

/* Message of the calling thread's most recent failure ("" if none). */
const char* llg_last_error(void);

/* Library version string. */
const char* llg_version(void);

/* Create a solver for one problem (Methods, micromagnetic simulations: the
 * nodal finite-difference discretisation of Eq. 11 with the Zeeman, demag and
 * exchange fields, plus uniaxial anisotropy): validates the parameters,
 * allocates the workspace on the current HIP device, builds the Newell tensor
 * of the cell (float64 on the host) and its Fourier spectrum on the padded
 * grid, and copies the masks.  Blocks the host.
 * Errors: LLG_EINVAL (bad parameter), LLG_ESHAPE (grid larger than the FFT
 * kernels support, or a spectrum of 4 GiB or more: the kernels address it at
 * 32-bit byte offsets), LLG_ENOMEM, LLG_EHIP. */
int llg_create(const llg_problem* p, const llg_masks* masks, llg_handle** out);

/* Free the handle and its workspace (synchronises the device).  NULL is a
 * no-op.  (Lifetime only; no passage of the method.) */
int llg_destroy(llg_handle* h);

/* Material map of the level set (Eq. 4 and the paragraph after it):
 *   psi_i = D_i / (1 + exp(-a phi_i)) + (1 - D_i) psi_fixed_i,
 * D = design mask of the handle.  phi has nx*ny entries when extrude_z != 0
 * (one 2D level set repeated through the thickness), else N.  psi_fixed and
 * psi_out have N entries.  Ms, A and K of a node scale with its psi. */
int llg_levelset_to_Ms(llg_handle* h, const void* phi, const void* psi_fixed, double a, int extrude_z,
                       void* psi_out, hipStream_t stream);

/* Chain rule through the map above: dJdphi = D a H (1 - H) dJdpsi, summed over
 * z when extrude_z != 0.  dJdpsi (N) and dJdphi_out (nx*ny or N) are float64. */
int llg_levelset_to_Ms_vjp(llg_handle* h, const void* phi, const double* dJdpsi, double a, int extrude_z,
                           double* dJdphi_out, hipStream_t stream);

/* Effective field B (T, 3N) at the state m (3N) and time t, from the enabled
 * terms (Methods: Zeeman with the drive at t, demag, exchange; anisotropy),
 * with Ms, A and K scaled by psi (the paragraph after Eq. 4); the LL
 * right-hand side of Eq. 11, dm/dt (3N), too if rhs_out is not NULL.
 * Nodes with psi = 0 have dm/dt = 0.  psi (N) and m are device arrays of the
 * handle's precision, component-major (all x, then all y, then all z). */
int llg_field(llg_handle* h, const void* psi, const void* m, double t, void* B_out, void* rhs_out,
              hipStream_t stream);

/* Integrate n_steps classic RK4 steps of the LL form of Eq. 11 from m0 (3N) at
 * time t0 (step n runs from t0 + n dt).  Writes m(t0 + n_steps dt) to m_out
 * (may alias m0).  Records what llg_adjoint needs (psi, t0, n_steps,
 * checkpoints per the handle's policy).  If obj is a port objective its
 * running cost is accumulated and written to *J_dev (device double) at the
 * end; J_dev may be NULL otherwise.  1 <= n_steps <= max_steps.
 * Errors: LLG_EINVAL, LLG_ENOMEM (checkpoint capacity), LLG_EHIP. */
int llg_forward(llg_handle* h, const void* psi, const void* m0, double t0, int64_t n_steps,
                const llg_objective_spec* obj, void* m_out, double* J_dev, hipStream_t stream);

/* Terminal objective at the state m (3N) (the objectives of the Results
 * sections; t is the time of m, which the Zeeman energy of a driven run
 * needs): for LLG_OBJ_ENERGY_AREA writes J to
 * *J_dev, dJ/dm to dJdm_out (3N, handle precision) and the explicit dJ/dpsi
 * to dJdpsi_out (N, float64); energies_dev (device double[5]: exchange, demag,
 * Zeeman at t, anisotropy, total; J) receives the energy terms when not NULL.
 * For LLG_OBJ_PORT_MY2, LLG_OBJ_PORT_SPECTRAL and LLG_OBJ_MAG_CURVE the objective is a function of
 * the trajectory: J_dev receives the value the last llg_forward computed,
 * dJdm_out and dJdpsi_out are zeroed (its sources are injected by llg_adjoint;
 * for the spectral and curve objectives they are those of the last
 * llg_forward's frequencies, targets and weights). */
int llg_objective(llg_handle* h, const llg_objective_spec* obj, const void* psi, const void* m, double t,
                  double* J_dev, void* dJdm_out, double* dJdpsi_out, double* energies_dev, hipStream_t stream);

/* Discrete adjoint of the last llg_forward on this handle (same psi, same
 * stream order).  Starts from lambda_N = dJdm_T (+ the port source at n_steps)
 * and walks the RK4 steps backwards, recomputing checkpointed segments; adds
 * dJdpsi_expl (may be NULL).  Writes dJ/dpsi (N, float64) to dJdpsi_out and,
 * if not NULL, dJ/dm0 (3N, handle precision) to dJdm0_out.
 * Errors: LLG_ESTATE (no forward recorded), LLG_EINVAL, LLG_EHIP. */
int llg_adjoint(llg_handle* h, const void* psi, const void* dJdm_T, const double* dJdpsi_expl,
                const llg_objective_spec* obj, double* dJdpsi_out, void* dJdm0_out, hipStream_t stream);

/* Size and centre-of-mass constraints of the regularised objective (Eq. 9):
 *   J = xi (S - S_target)^2 + nu (|x_c - x0| + |y_c - y0|),
 * S = sum_i psi_i / nz (in-plane area in cells), x_c = sum_i psi_i x_i / sum_i psi_i,
 * y_c likewise (node indices).  psi: device, N entries in the handle's precision.
 * Writes J to *J_dev (device double) and, if dJdpsi_out (device, N doubles) is
 * not NULL, dJ/dpsi there, ready to pass as dJdpsi_expl to llg_adjoint (the
 * constraints depend on psi only).  |.| takes the zero subgradient at 0; with no
 * material the centre term is 0.  Single-instance handles; uses a small scratch
 * buffer of the handle (allocated on first use), so calls on one handle and
 * stream are ordered.  Errors: LLG_EINVAL, LLG_ENOMEM, LLG_EHIP. */
int llg_shape_penalty(llg_handle* h, const void* psi, double xi, double S_target, double nu, double x0, double y0,
                      double* J_dev, double* dJdpsi_out, hipStream_t stream);

/* llg_shape_penalty for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and results, but its block partial sums live in a
 * static device array of the library (one per GPU, 786 496 bytes, held until
 * the process ends) instead of the handle's scratch, which llg_shape_penalty
 * allocates on its first call.  Nothing is allocated: the array's device
 * address is looked up once per device.  At most 8 388 608 nodes (2^23);
 * larger grids return LLG_ENOMEM before any device work.  Every call on a GPU
 * uses that GPU's one array and nothing in it carries over between calls (each
 * call writes what it reads), but calls that overlap in time on one GPU (other
 * streams, other threads) race on it: order them on one stream. */
int llg_shape_penalty_noalloc(llg_handle* h, const void* psi, double xi, double S_target, double nu, double x0,
                              double y0, double* J_dev, double* dJdpsi_out, hipStream_t stream);

/* ---- adaptive integration --------------------------------------------
 * The Methods integrate adaptively: embedded Dormand-Prince 5(4) steps (fifth
 * order carried, fourth order for the estimate) from m0 at t0 to exactly t_end,
 * first trial step h0.  A trial is accepted when max over all nodes and
 * components of |y5 - y4| / (atol + rtol max(|y_n|, |y5|)) <= 1; the next step
 * is h min(5, max(0.2, 0.9 err^(-1/5))), without growth right after a
 * rejection.  Every accepted state is kept (at most max_steps accepted steps,
 * else LLG_ENOMEM), so that llg_adjoint_adaptive can transpose the accepted
 * steps with their sizes held fixed.  The controller reads each error norm on
 * the host (the call blocks per trial step).  Single-instance handles; the
 * stage store must hold 6 stage states (checkpoint K x halves >= 6, true for
 * max_steps >= 36).  m_out (nullable, 3N) receives m(t_end); n_accepted /
 * n_rejected (nullable, host) the step counts.
 * Errors: LLG_EINVAL, LLG_ENOMEM, LLG_ENOTSUP, LLG_ENONFINITE, LLG_EHIP. */
int llg_forward_adaptive(llg_handle* h, const void* psi, const void* m0, double t0, double t_end, double h0,
                         double rtol, double atol, void* m_out, int64_t* n_accepted, int64_t* n_rejected,
                         hipStream_t stream);

/* With keep != 0, later llg_forward_adaptive runs also keep every accepted
 * step's stage states and fields (11 state vectors of 3N per step, a device
 * store of (max_steps + 1) x 11 x 3N elements, allocated by the first such
 * run), and llg_adjoint_adaptive reads them instead of recomputing six field
 * evaluations per step.  The results are bitwise the same either way.  With
 * keep == 0 (the default) runs keep only the accepted states; an allocated
 * store stays until llg_destroy.  Single-instance handles.
 * Errors: LLG_EINVAL (NULL handle or a batch); LLG_ENOMEM at the next run. */
int llg_set_keep_stages(llg_handle* h, int keep);

/* Accepted step sizes of the last llg_forward_adaptive (host array of cap >= n_accepted). */
int llg_adaptive_steps(const llg_handle* h, double* hs_out, int64_t cap);

/* Discrete adjoint of the last adaptive run with its step sizes fixed: from
 * lambda_N = dJdm_T (3N; NULL = 0), per step kappa_s = h (b_s lambda' + sum_{i>s}
 * a_is mu_i), mu_s = J_f(Y_s)^T kappa_s (stages recomputed from the kept state,
 * or read from the stage store, see llg_set_keep_stages),
 * lambda = lambda' + sum_s mu_s; dJ/dpsi accumulates kappa_s . df/dpsi(Y_s) and
 * dJdpsi_expl (nullable).  Writes dJ/dpsi (N, float64) and, if not NULL, dJ/dm0
 * (3N).  A terminal objective is evaluated with llg_objective on m(t_end).
 * Errors: LLG_ESTATE (no adaptive run), LLG_EINVAL, LLG_EHIP. */
int llg_adjoint_adaptive(llg_handle* h, const void* psi, const void* dJdm_T, const double* dJdpsi_expl,
                         double* dJdpsi_out, void* dJdm0_out, hipStream_t stream);

/* Continuous adjoint (Eqs. 6-7), for comparison with the discrete one: the
 * adjoint equation da/dt = -J_f(m)^T a and dJ/dpsi = integral a . df/dpsi are
 * integrated backwards over every interval of the last llg_forward_adaptive
 * run, each split into n_sub (1..64) equal classic RK4 steps, with the
 * Jacobians taken at states of the cubic Hermite interpolant of the kept
 * states and their rates (not at the forward stage states).  Otherwise the
 * same arguments and outputs as llg_adjoint_adaptive.  The result differs
 * from the discrete gradient by the discretisation error of the backward
 * integration (fourth order in the step).  On stiff runs the adaptive steps
 * lie at the edge of Dormand-Prince's stability region, beyond RK4's: n_sub = 1
 * then diverges (non-finite output in FP32) and n_sub = 2 is needed.
 * LLG_EINVAL for n_sub outside 1..64, LLG_ESTATE without an adaptive run. */
int llg_adjoint_continuous(llg_handle* h, const void* psi, const void* dJdm_T, const double* dJdpsi_expl, int n_sub,
                           double* dJdpsi_out, void* dJdm0_out, hipStream_t stream);

/* Device bytes the checkpoint store needs for n_steps under a policy
 * (snapshots + recomputed stage states), without allocating anything.  The
 * adjoint of Eqs. 6-7 runs backwards over the forward trajectory, which is
 * stored (ALL) or recomputed from snapshots (SQRT, BINOMIAL).  It takes the
 * problem rather than a handle so that a caller can size the store, and pick
 * a policy, before creating the handle that would allocate it. */
int llg_query_memory(const llg_problem* p, int64_t n_steps, int32_t policy, int32_t ckpt_param, size_t* bytes);

/* Forward RK4 steps that llg_adjoint recomputes after a forward run of n_steps
 * under a checkpoint policy (host only; n_steps for SQRT and ALL). */
int llg_query_recompute(int64_t n_steps, int32_t policy, int32_t ckpt_param, int64_t* steps);

/* HIP graphs (default off).  While enabled, the launch sequence of
 * llg_forward / llg_adjoint (and their batch forms) is captured into a HIP
 * graph on the first call with a given signature (n_steps, t0, objective kind
 * and window, adjoint inputs present) and replayed on later calls, on a stream
 * of the handle ordered after the caller's stream (event fork/join), so no
 * per-launch host work remains.  Up to 8 graphs are cached per handle; the
 * copies of the caller's arrays in and out stay ordinary stream operations.
 * Disabling synchronises the handle's graph stream and frees the graphs.
 * Profiling (llg_profile) runs the sequences without graphs, and so do calls
 * of more than 2 000 RK4 steps (graphs of that many nodes are not supported);
 * either way the results are the same bits.
 * Errors: LLG_EINVAL (NULL handle), LLG_EHIP (capture or instantiation failed). */
int llg_set_graphs(llg_handle* h, int enable);

/* Launch configuration of a handle's kernels (one for all instances of a
 * batch), 8 ints:
 *   cfg[0] column tile (x-bins per column-kernel block: 1, 2, 4, 8 or 16),
 *   cfg[1] column-kernel threads, cfg[2] its largest FFT radix,
 *   cfg[3] forward row-kernel threads, cfg[4] its largest FFT radix,
 *   cfg[5] backward row-kernel threads, cfg[6] its largest FFT radix,
 *   cfg[7] node values per row the backward row kernel stages in LDS
 *          (4: field adjoint and psi; 7: also the stage state).
 * Threads are multiples of 64; radices are 4, 8, or 16 (float only): a
 * smaller radix spreads a transform over more lanes, a larger one needs fewer
 * passes.  For given radices every tiling computes identical bits; another
 * radix changes only the rounding order of the transforms.
 * llg_set_launch_config validates (LLG_EINVAL / LLG_ESHAPE when a tile does
 * not fit 160 KiB of LDS or the FFT register budget), synchronises the device
 * and drops cached graphs. */
int llg_launch_config(const llg_handle* h, int32_t cfg[8]);
int llg_set_launch_config(llg_handle* h, const int32_t cfg[8]);

/* Autotuner: times the column kernel over every valid (tile, threads) pair
 * and one forward plus one backward row-kernel stage over the valid row block
 * sizes, on the handle's own buffers, and keeps the fastest configuration.
 * Blocks the host; overwrites the handle's state buffers, so the record of the
 * last llg_forward is dropped (call it after create, before forward).
 * Errors: LLG_EINVAL (NULL handle), LLG_EHIP. */
int llg_autotune(llg_handle* h, hipStream_t stream);

/* Kernel classes reported by the profiling counters. */
#define LLG_KIND_STAGE_FWD 0 /* forward local kernel: row FFTs + fields + LL RHS + RK4 stage */
#define LLG_KIND_COLUMN 1    /* column kernel: y/z FFTs and tensor-spectrum multiply       */
#define LLG_KIND_STAGE_BWD 2 /* backward local kernel of the discrete adjoint              */
#define LLG_KIND_COUNT 3

/* Profiling: llg_profile(h, k) with k > 0 brackets every k-th launch of each
 * kernel class (k = 1: every launch) by two HIP events bound to the dispatch
 * on the call's stream; k = 0 stops.  llg_profile_read synchronises on the
 * recorded events and returns, for one kernel class, the summed device time
 * (ms), the number of bracketed launches, and the algorithmic HBM bytes of
 * those launches (every array element the kernel must read or write counted
 * once).  reset != 0 clears the class's totals after reading.
 * llg_profile(h, 1) returns LLG_ENOTSUP while a profiler collects hardware
 * counters from the process (ROCPROF_COUNTER_COLLECTION set, as rocprofv3
 * --pmc does): event-timed dispatches are not combined with counter
 * collection, under which one run crashed in the HIP launch path. */
int llg_profile(llg_handle* h, int enable);
int llg_profile_read(llg_handle* h, int32_t kind, double* ms, int64_t* launches, double* bytes, int reset);

/* The demagnetising tensor the library builds the dipole-dipole field term
 * from (Methods: the effective field's demagnetising part), host only, float64:
 * the cell-averaged tensor N(r) = (1/V) int T(s) D(r + s) ds between two cells
 * of edges dx, dy, dz (m) whose centres are (X, Y, Z) apart, with
 * T(s) = prod_d (h_d - |s_d|)_+ and D(p) = -(3 p p^T / |p|^2 - I) / (4 pi |p|^3);
 * the mean field in one cell is -N(r) M of the other's uniform M.
 * out[6] = N_xx, N_yy, N_zz, N_xy, N_xz, N_yz.  method 0: what the library uses
 * (Newell, Williams & Dunlop's closed form for centres less than two largest
 * cell edges apart, Gauss-Jacobi quadrature of the tent integral beyond);
 * 1: the closed form at any offset; 2: the quadrature (centres at least two
 * largest edges apart).  No device work.  Errors: LLG_EINVAL. */
int llg_demag_tensor(double dx, double dy, double dz, double X, double Y, double Z, int32_t method, double* out);

/* Padded FFT sizes the handle uses (Px, Py, Pz); of the first instance of a batch. */
int llg_fft_sizes(const llg_handle* h, int32_t* P3);

/* ---- RBF level set and the amplitude update ----------------------------
 * The level set as a function of RBF amplitudes s (n_rbf of them), handle-free.
 * Eq. 2: cone g_i(x, y) = s_i - sqrt((x - x_i)^2 + (y - y_i)^2 + c^2), with x, y
 * node indices (x = ix, y = iy) and c in the same units.  Eq. 3: on the design
 * region Phi = [sum_i (g_i + dphi)^p]^(1/p) - dphi, dphi = |smallest g_i on the
 * design region|; then (the paragraph after Eq. 3) Phi is renormalised into
 * [-1, 1] by dividing by its largest magnitude on the design region when
 * normalize != 0.  Phi = 0 off the design region.  All pointers are device
 * pointers; centers holds 2 n_rbf doubles (x_0..x_{n-1}, then y_0..y_{n-1}), s
 * n_rbf doubles, design nx*ny bytes (row-major, x fastest; non-zero = design).
 * Outputs are written on `stream`; nothing is allocated.  Results depend only
 * on the inputs and the sizes (fixed reduction orders).
 * Errors: LLG_EINVAL (NULL pointer, dtype, p < 1, n_rbf outside 1..131072,
 * non-finite c), LLG_ESHAPE (nx*ny outside 1..2^30), LLG_EHIP. */

/* Doubles of device workspace that llg_rbf_levelset and llg_rbf_levelset_vjp
 * need for this size (the caller allocates it; one buffer serves both calls). */
int llg_rbf_work_len(int32_t nx, int32_t ny, int32_t n_rbf, int64_t* len);

/* Phi (nx*ny, dtype) from s.  pnorm_out (nullable, nx*ny, dtype) receives the
 * p-norm S = Phi_raw + dphi that the VJP needs.  On return work[0] = dphi and
 * work[1] = the renormalisation factor (1 / max |Phi_raw|, or 1); the VJP reads
 * both from the same buffer. */
int llg_rbf_levelset(int32_t dtype, int32_t nx, int32_t ny, int32_t n_rbf, const double* centers, const double* s,
                     double c, double p, const uint8_t* design, int normalize, void* phi_out, void* pnorm_out,
                     double* work, hipStream_t stream);

/* dJ/ds (n_rbf doubles) from dJ/dPhi (nx*ny doubles, as llg_levelset_to_Ms_vjp
 * writes it):  dJ/ds_i = f sum_x dJ/dPhi(x) ((g_i(x) + dphi) / S(x))^(p - 1)
 * over design nodes, with dphi, f (work[0], work[1]) and S (pnorm) from the
 * llg_rbf_levelset call on the same s: the shift and the scale are held fixed. */
int llg_rbf_levelset_vjp(int32_t dtype, int32_t nx, int32_t ny, int32_t n_rbf, const double* centers,
                         const double* s, double c, double p, const uint8_t* design, const double* dJdphi,
                         const void* pnorm, double* work, double* dJds_out, hipStream_t stream);

/* Device time of the RBF pair kernels (process-wide, all streams): with
 * profiling on, every launch of the kinds below carries a start/end event
 * pair bound to its dispatch; llg_rbf_profile_read synchronises on the
 * recorded events and returns the summed milliseconds, the launch count and
 * the node-RBF pairs (nx*ny*n_rbf per launch) of a kind since the last reset. */
#define LLG_RBF_KIND_CONES 0 /* pass 1: largest cone per node, smallest cone per block */
#define LLG_RBF_KIND_PNORM 1 /* pass 2: max-scaled p-norm per node                    */
#define LLG_RBF_KIND_VJP 2   /* dJ/ds partial sums over node chunks                   */
#define LLG_RBF_KIND_COUNT 3
int llg_rbf_profile(int enable); /* LLG_ENOTSUP under counter collection, as llg_profile */
int llg_rbf_profile_read(int32_t kind, double* ms, int64_t* launches, double* pairs, int reset);

/* One Adam step on n device doubles, in place (the amplitude update of Eq. 5
 * with Adam's adaptive moments, Kingma & Ba's Algorithm 1 with bias
 * correction): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 * s -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).  t >= 1 counts
 * steps; m and v start at zero.  Errors: LLG_EINVAL, LLG_EHIP. */
int llg_adam_step(int32_t n, double* s, const double* grad, double* m, double* v, int64_t t, double lr, double beta1,
                  double beta2, double eps, hipStream_t stream);

/* ---- batched execution ------------------------------------------------
 * Many level-set designs and drive frequencies, on grids of different sizes,
 * integrated together (the optimisation sweep of many initial level sets at
 * once).  Instances must share dtype, terms, dt, max_steps and the checkpoint
 * policy; grid, cell, material, field and drive parameters may differ.  The
 * pointer arguments are HOST arrays of n device pointers (one per instance,
 * sized for that instance as in the single-instance call); an array argument
 * documented as nullable may be NULL as a whole.  J_dev receives n doubles.
 * Results per instance are identical to running that instance alone. */
int llg_batch_create(const llg_problem* probs, const llg_masks* masks, int32_t n, llg_batch** out);
int llg_batch_destroy(llg_batch* b);
int llg_batch_size(const llg_batch* b, int32_t* n);
int llg_batch_levelset_to_Ms(llg_batch* b, const void* const* phi, const void* const* psi_fixed /* nullable */,
                             double a, int extrude_z, void* const* psi_out, hipStream_t stream);
int llg_batch_levelset_to_Ms_vjp(llg_batch* b, const void* const* phi, const double* const* dJdpsi, double a,
                                 int extrude_z, double* const* dJdphi_out, hipStream_t stream);
int llg_batch_forward(llg_batch* b, const void* const* psi, const void* const* m0, double t0, int64_t n_steps,
                      const llg_objective_spec* obj, void* const* m_out /* nullable */, double* J_dev /* nullable */,
                      hipStream_t stream);
int llg_batch_adjoint(llg_batch* b, const void* const* psi, const void* const* dJdm_T /* nullable */,
                      const double* const* dJdpsi_expl /* nullable */, const llg_objective_spec* obj,
                      double* const* dJdpsi_out, void* const* dJdm0_out /* nullable */, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LLG_H */
