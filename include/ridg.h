/*
 * ridg.h - C ABI of the MI355X RIDG (regionally-implicit discontinuous Galerkin)
 * predictor/corrector library (libridg.so, HIP kernels for gfx950).
 *
 * Method (arXiv 2101.01231): scalar conservation law q_t + div(v q) = 0
 * (Sec. 2.1) on a uniform periodic Cartesian mesh of the box
 * [0,L_1] x .. x [0,L_d] (the unit box by default), d = 1, 2, 3. Each step has two stages:
 *   prediction (Sec. 2.2, eq. pred_full_system): for every element, the
 *     space-time DG system on its region of 3^d vertex neighbours (upwind
 *     fluxes on faces inside the region, the region element's own trace on
 *     the region boundary, causal source from the state at t^n) is solved and
 *     only the centre's space-time coefficients W are kept;
 *   correction (Sec. 2.3): explicit flux-form update of every element's
 *     modal coefficients from its own W and its face neighbours' W
 *     (Rusanov flux, which for linear advection is exact upwinding).
 * Region matrices are assembled quasi-quadrature-free (Sec. 3): the velocity
 * is projected on the space-time basis and contracted with exact,
 * precomputed Legendre triple-product tensors.
 *
 * Basis: orthonormal (w.r.t. the element average) scaled Legendre products of
 * total degree <= order-1 in space (theta = C(order-1+d, d) modes) and in
 * space-time (theta_T = C(order+d, d+1) modes).
 *
 * State layout (set/get): q[e * theta + k], element e = i0 + n0 (i1 + n1 i2)
 * (x fastest), mode k ordered by total degree, then lexicographically
 * descending in the exponents (a_1, ..., a_d): in 2D, order 3:
 * 1, x, y, x^2, xy, y^2. Prediction layout (ridg_get_prediction):
 * w[e * theta_T + k] with space-time exponents (b_t, b_1..b_d) ordered the
 * same way (time exponent first).
 *
 * Conventions: every function returns 0 (RIDG_OK) on success, a negative
 * RIDG_E_* code on error (the handle is left unchanged and
 * ridg_last_error() describes the failure), or a positive RIDG_W_* warning
 * (the call still did its work). All device work goes to the HIP stream
 * given at creation; calls on one handle must not overlap from several host
 * threads. Handles are independent of each other.
 */
#ifndef RIDG_H_
#define RIDG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RIDG_ABI_VERSION 3

/* return codes */
#define RIDG_OK 0
#define RIDG_E_INVAL (-1)       /* bad argument: dims, sizes, dt, null pointer, count mismatch */
#define RIDG_E_NOMEM (-2)       /* workspace smaller than ridg_workspace_bytes() */
#define RIDG_E_DEVICE (-3)      /* a HIP call failed (message in ridg_last_error) */
#define RIDG_E_SINGULAR (-4)    /* zero pivot in a host FP64 factorisation */
#define RIDG_E_NONFINITE (-5)   /* NaN/Inf in the input state */
#define RIDG_E_UNSUPPORTED (-6) /* valid problem outside what the library implements */
#define RIDG_W_UNSTABLE 1       /* constant velocity: the step's von Neumann amplification exceeds 1
                                   (ridg_info.spectral_radius > 1 + 1e-10); affine velocity: the CFL
                                   number dt max|v_i|/h_i exceeds 1 */
#define RIDG_W_NOT_CONVERGED 2  /* RIDG_FLUX_BURGERS (ridg_get_state): the Newton iteration of at least one
                                   region stopped at newton_max_iter without meeting its tolerance since
                                   the handle was created or ridg_newton_stats last reset the counters (the
                                   time step is too large for the local compression of the solution) */

/* velocity field kinds */
#define RIDG_FLUX_CONST 0    /* v = velocity[0..d-1] */
#define RIDG_FLUX_ROTATION 1 /* 2D solid-body rotation v = (-(y - c_y), x - c_x), c = rot_center */
#define RIDG_FLUX_AFFINE 2   /* v_i = velocity[i] + sum_j vel_grad[3 i + j] x_j, vel_grad[3 i + i] = 0 */
#define RIDG_FLUX_BURGERS 3  /* nonlinear: q_t + sum_i (q^2/2)_{x_i} = 0 (eq. burger2d; the same flux along
                                every axis). Prediction: Newton iterations on each region system (Sec. 3),
                                starting from Q^n held constant in time, Jacobian volume term assembled
                                quasi-quadrature-free (F'(w) projected on the space-time basis, exact
                                Legendre triple products), face terms by Gauss quadrature; stop when
                                max|delta| <= 1e-13 max(1, max|W|). Rusanov flux with the wave speed
                                max(|mean q_a|, |mean q_b|) of the two elements' states at t^n inside the
                                region and in the correction; own-trace physical flux on the region
                                boundary. FP64; orders 1-5 in 1D, 1-4 in 2D, 1-2 in 3D; velocity fields
                                are ignored */

/* basis families (Sec. 2.1) */
#define RIDG_BASIS_P 0 /* total degree <= order-1 in space and in space-time */
#define RIDG_BASIS_Q 1 /* tensor degree <= order-1 per variable (the paper's space, Sec. 2.1-2.2): theta =
                          order^d, theta_T = order^(d+1), same mode ordering rule. Constant velocity, FP64,
                          1D (orders 1-12) and 2D (orders 1-5); the step runs as the composite stencil
                          (RIDG_OPT_COMPOSITE is always on, the other options and ridg_get_prediction,
                          ridg_step_batch, ridg_autotune and ridg_advance_static give RIDG_E_UNSUPPORTED) */

/* arithmetic of the prediction (the correction is always FP64) */
#define RIDG_FP64 0
#define RIDG_FP32_REFINE 1 /* REGION: FP32 block solves + FP64-residual iterative refinement (refine_steps
                              sweeps). PREFACTORED (3D, orders 2-3, n[0] % 16 == 0, n[1] % 4 == 0,
                              n[2] % 4 == 0): predictions on the matrix cores with FP32 operands and FP32
                              accumulation (no solve to refine: refine_steps is ignored), FP64 correction */

/* region solver */
#define RIDG_SOLVER_AUTO 0        /* PREFACTORED for RIDG_FLUX_CONST, REGION otherwise */
#define RIDG_SOLVER_PREFACTORED 1 /* constant v only: W = G Q_region with G = E_c A^-1 C from a host FP64 LU */
#define RIDG_SOLVER_REGION 2      /* per element: assemble (QQF) and solve the region system by upwind block
                                     elimination, Gauss-Jordan with partial pivoting per block; regions whose centre lies on
                                     a dependency cycle tear one block (multi-right-hand-side elimination plus
                                     one block-sized system), else use the dense path */
#define RIDG_SOLVER_DENSE 3       /* per element: dense pivoted LU of the whole 3^d theta_T region system */
#define RIDG_SOLVER_NEWTON 4      /* RIDG_FLUX_BURGERS (its only solver; AUTO selects it): one workgroup per
                                     region runs the Newton iterations, each a dense pivoted elimination of
                                     the whole region Jacobian in LDS (FP64 up to 48 KB, FP32 above; the
                                     residual is always FP64, so the iteration converges to the FP64 root) */

/* memory kinds for set/get */
#define RIDG_HOST 0
#define RIDG_DEVICE 1

typedef struct ridg_problem {
  int32_t dim;          /* d in {1, 2, 3} */
  int32_t n[3];         /* elements per axis, n[i] >= 3 for i < dim (the 3^d region elements are distinct) */
  int32_t order;        /* M >= 1: basis of degree M-1; the library implements M <= 5 (tensor basis in 1D: M <= 12) */
  int32_t basis;        /* RIDG_BASIS_P (default) or RIDG_BASIS_Q */
  int32_t flux;         /* RIDG_FLUX_* */
  int32_t newton_max_iter; /* RIDG_FLUX_BURGERS: Newton iterations per region at most (0: 20; <= 100);
                              must be 0 for the linear fluxes */
  double velocity[3];   /* CONST: v; AFFINE: constant part */
  double rot_center[2]; /* ROTATION: centre; must lie on element boundaries (c_x / h_x, c_y / h_y integers) */
  double vel_grad[9];   /* AFFINE: row-major dv_i/dx_j, diagonal must be 0 */
  double length[3];     /* box side lengths L_i > 0 (h_i = L_i / n_i); 0 stands for 1 */
  int32_t precision;    /* RIDG_FP64 or RIDG_FP32_REFINE */
  int32_t refine_steps; /* FP32_REFINE: refinement sweeps 0..3 */
  int32_t solver;       /* RIDG_SOLVER_* */
  int32_t reserved;     /* must be 0 */
} ridg_problem;

typedef struct ridg_info {
  int32_t abi_version;
  int32_t theta;      /* spatial modes per element */
  int32_t theta_t;    /* space-time modes per element */
  int32_t solver;     /* resolved RIDG_SOLVER_* */
  int64_t n_elements;
  int64_t n_plans;          /* REGION: distinct upwind elimination plans */
  int64_t n_tear_elements;  /* REGION: regions on a dependency cycle solved by tearing one block */
  int64_t n_dense_elements; /* REGION: regions solved by dense LU of the whole region */
  int64_t n_taps;           /* PREFACTORED: non-zero blocks of G (upwind cone) */
  /* Algorithmic flops per step (FMA = 2) of the method as the library decomposes it, not instruction
   * counts: PREFACTORED, the tap products; REGION, per solved block the QQF assembly, the upwind
   * couplings and an LU-equivalent solve (2/3 theta_T^3 + 2 theta_T^2; the Gauss-Jordan kernels
   * execute about 1.5x the elimination part); DENSE, LU of the whole region. Correction: the volume
   * and face terms of Sec. 2.3 term by term (constant velocity: the precombined tap products). */
  double flops_predict;     /* per step, prediction (RIDG_SOLVER_NEWTON: per Newton iteration of every
                               region: Jacobian and residual assembly plus the dense elimination) */
  double flops_correct;     /* per step, correction */
  double bytes_predict;     /* per step, prediction: algorithmic HBM bytes (state in, predictions out) */
  double bytes_correct;     /* per step, correction: state in/out, predictions in */
  double flops_composite;   /* PREFACTORED with RIDG_OPT_COMPOSITE: per step */
  double bytes_composite;   /* PREFACTORED with RIDG_OPT_COMPOSITE: state in/out per step */
  int32_t basis;            /* RIDG_BASIS_* */
  int32_t reserved;
  /* 0 until a step of some dt has been analysed: */
  double spectral_radius;     /* constant velocity: von Neumann amplification at the dt of the last ridg_step */
  double static_pivot_growth; /* REGION: growth factor measured for static pivots (layout 5) at the dt of
                                 the last ridg_step or ridg_get_prediction */
} ridg_info;

/* Accumulated stage times of ridg_step, from HIP events recorded on the handle's stream. */
typedef struct ridg_timing {
  int64_t steps;     /* steps timed since the last ridg_get_timing */
  double predict_ms; /* sum over steps: prediction kernels (region gather, assembly, solve) */
  double correct_ms; /* sum over steps: correction kernel */
  double max_step_ms; /* slowest single step (prediction + correction) */
} ridg_timing;

typedef struct ridg_handle ridg_t;

/* Size in bytes of the device workspace ridg_create needs for this problem.
 * Pure host function (no device calls); validates the problem. */
int ridg_workspace_bytes(const ridg_problem* problem, size_t* bytes);

/* Create a handle. d_workspace: device memory of at least ws_bytes =
 * ridg_workspace_bytes(), allocated by the caller, 256-byte aligned, owned by
 * the caller and borrowed until ridg_destroy. hip_stream: a hipStream_t (NULL
 * = the default stream) on which all work of this handle is queued. Host-side
 * FP64 precompute (exact reference tensors, elimination plans, prefactored
 * operators) happens here. The state is zero after creation. */
int ridg_create(const ridg_problem* problem, void* d_workspace, size_t ws_bytes, void* hip_stream,
                ridg_t** out);

/* Copy a state in (layout above). count must equal n_elements * theta. where:
 * RIDG_HOST (pageable host memory; the call returns after the copy) or
 * RIDG_DEVICE (device memory; queued on the stream). Non-finite host values
 * give RIDG_E_NONFINITE and leave the state unchanged. */
int ridg_set_state(ridg_t* h, const double* q, size_t count, int32_t where);

/* Queue n_steps >= 0 RIDG steps of size dt > 0 on the stream (asynchronous).
 * dt-dependent host tables are rebuilt when dt changes (for a constant velocity this includes the
 * von Neumann analysis of the composed step: eigenvalues of the amplification matrix on a grid of
 * wavenumbers, 256 points in 1D, 48^2 in 2D, 12^3 in 3D). Returns RIDG_W_UNSTABLE (the steps are
 * still queued) when that amplification exceeds 1 + 1e-10, or, for an affine velocity, when the CFL
 * number dt max|v_i| / h_i exceeds 1. */
int ridg_step(ridg_t* h, int32_t n_steps, double dt);

/* Copy the state out (layout above); synchronises the stream for RIDG_HOST. RIDG_FLUX_BURGERS: returns
 * RIDG_W_NOT_CONVERGED (after the copy) when a Newton failure has been counted (RIDG_HOST only). */
int ridg_get_state(ridg_t* h, double* q, size_t count, int32_t where);

/* The centre predictions W of the current state for step size dt, without the
 * correction (count = n_elements * theta_T, layout above). */
int ridg_get_prediction(ridg_t* h, double dt, double* w, size_t count, int32_t where);

/* Sizes and cost model of the handle. */
int ridg_get_info(ridg_t* h, ridg_info* info);

/* Switch stage timing on (1) or off (0). When on, ridg_step records a HIP event before the
 * prediction, between prediction and correction, and after the correction of every step. */
int ridg_enable_timing(ridg_t* h, int32_t on);

/* Synchronise the stream and return (and reset) the accumulated stage times. */
int ridg_get_timing(ridg_t* h, ridg_timing* out);

/* Execution options (all default 0). Values are 0 or 1 unless stated.
 *   RIDG_OPT_GRAPH: replay a captured HIP graph of two steps instead of launching kernels one by
 *     one (recaptured when dt or an option changes; not used while stage timing is on).
 *   RIDG_OPT_PLAN_LAYOUT (REGION): 0 = theta_T-lane segments packed in the wavefront, 1 = segments
 *     padded to a power of two (DPP reductions), 2 = two regions per packed segment with their
 *     eliminations interleaved, 3 = two rows per lane (half-width segments; each published pivot
 *     row is read once for two rows), 4 = up to three rows per lane in power-of-two segments
 *     (DPP pivot reductions). 2 to 4 are RIDG_FP64 only and give bitwise the results of 0 and 1.
 *     5 = the geometry of 4 with static pivots (row c pivots column c, no row exchanges, the next
 *     pivot row published from registers): FP64 or RIDG_FP32_REFINE. It runs where the host has
 *     measured elimination in natural order to be stable for the problem's velocity range at the
 *     step's dt (growth factor <= 64 on every diagonal block form); otherwise the step falls back
 *     to layout 4 (FP64) or 1 (RIDG_FP32_REFINE). Results agree with the other layouts to rounding.
 *   RIDG_OPT_FUSED (PREFACTORED, meshes whose state and predictions fit in 160 KB of LDS): run all
 *     n_steps of a ridg_step call in one single-workgroup kernel. */
#define RIDG_OPT_GRAPH 1
#define RIDG_OPT_PLAN_LAYOUT 2
#define RIDG_OPT_FUSED 3
#define RIDG_OPT_COMPOSITE 4 /* PREFACTORED: prediction and correction composed into one stencil on the
                                state, K_o = sum D_t G_s (the predictions are not stored). 2: the same stencil
                                marched along z by 16 x 16 tiles with three state planes in LDS (3D, orders
                                2-3, n[0], n[1] multiples of 16, n[2] a multiple of 8 or at most 64); bitwise
                                equal to 1. 3: four steps per launch, each 16 x 16 tile advancing the region
                                its result depends on in LDS (2D, FP64, n[0], n[1] multiples of 16; remaining
                                steps and timed steps run as 1); bitwise equal to 1 */
#define RIDG_OPT_MFMA 5      /* PREFACTORED: the prediction, correction or composite stencil as stacked-
                                right-hand-side products on the FP64 matrix cores */
#define RIDG_OPT_BRICK 6     /* PREFACTORED, 3D, orders 2-3, n[0] % 16 == 0, n[1] % 4 == 0, n[2] % 2 == 0: one
                                fused kernel per step on 16 x 4 x 2 bricks (state staged in LDS, predictions
                                of the brick and its upwind halo on the FP64 matrix cores, correction from
                                LDS). Always used by RIDG_FP32_REFINE PREFACTORED problems (FP32 products,
                                16 x 4 x 4 bricks) */
int ridg_set_option(ridg_t* h, int32_t option, int64_t value);
int ridg_get_option(ridg_t* h, int32_t option, int64_t* value);

/* Autotuner: time every applicable option set on `steps` steps of size dt (host clock around a
 * run synchronised with the handle's stream, lengthened up to 64x while it lasts under 2 ms; two
 * sweeps over the option sets, each set keeping its faster time), keep the fastest and restore the
 * state. Synchronises the stream. Results are cached per problem shape
 * in the process and, when the environment variable RIDG_AUTOTUNE_CACHE names a file, appended to
 * that file and reused by later processes (*best_ms_per_step is then -1). */
int ridg_autotune(ridg_t* h, double dt, int32_t steps, double* best_ms_per_step);

/* Serving: advance `count` handles by n_steps steps, handle i with step size dts[i], in shared
 * launches queued on hip_stream (the handles' own streams are not used; order calls on them with
 * ridg_synchronize or by using that same stream). When a handle's dt differs from the one its
 * earlier batched launches used, its operators are rebuilt after hip_stream has been synchronised
 * (those launches may still read them); the first batched call of a handle does not synchronise. Handles with the same dimension, order and
 * RIDG_OPT_MFMA setting share one prediction and one correction launch per step (up to 16 per
 * launch; the matrix-core or the vector kernels, as the option selects). Every handle must use
 * RIDG_SOLVER_PREFACTORED (constant velocity) on the same device and appear once; each state
 * advances exactly as ridg_step would advance it alone with RIDG_OPT_COMPOSITE off. */
int ridg_step_batch(ridg_t* const* handles, int32_t count, const double* dts, int32_t n_steps, void* hip_stream);

/* For callers that cannot allocate device memory (code under stream capture, serving loops with a
 * fixed memory plan): n_steps >= 0 steps of size dt > 0 of a constant-velocity FP64 problem
 * (RIDG_SOLVER_AUTO or RIDG_SOLVER_PREFACTORED), as ridg_create + ridg_set_state + ridg_step +
 * ridg_get_state would advance it with the default options, without a handle or a workspace.
 * q_in, q_out: device arrays in the state layout above (count = n_elements * theta; q_out may equal
 * q_in), owned by the caller. Queued on hip_stream (asynchronous; the host-side FP64 operator
 * precompute runs in the call and is cached per problem and dt). Intermediates (two states, the
 * predictions, the operators) live in a static per-device scratch array of 64 MiB: problems that
 * need more return RIDG_E_NOMEM before any device work. No device memory is allocated or freed.
 * Every call on one device shares that scratch: calls that overlap on a device (several host
 * threads or streams) race and must be serialised by the caller. */
int ridg_advance_static(const ridg_problem* problem, const double* q_in, double* q_out, size_t count,
                        int32_t n_steps, double dt, void* hip_stream);

/* RIDG_FLUX_BURGERS: Newton statistics of the steps (and predictions) queued since the handle was
 * created or the counters were last reset. Synchronises the stream. max_iters: the most iterations
 * any region took; total_iters: iterations summed over regions; solves: region solves run; failures:
 * regions that stopped at newton_max_iter without meeting the tolerance (their last iterate is used).
 * Any output pointer may be NULL. reset != 0 zeroes the counters after reading them.
 * RIDG_E_INVAL for the linear fluxes (Sec. 3: Newton's method on the prediction system). */
int ridg_newton_stats(ridg_t* h, int32_t* max_iters, int64_t* total_iters, int64_t* solves, int64_t* failures,
                      int32_t reset);

/* Assembly of the Newton Jacobian's volume flux block (Sec. 3: eq. Jacobian by quadrature, eq. Jacproj
 * and eq. Jacobian2 quasi-quadrature-free, and the perturbation method), for the Burgers flux
 * F(w) = w^2 / 2 on every axis, on n_elements space-time elements of dimension dim + 1 (orders 1..6,
 * total-degree basis, theta_T = C(order + dim, dim + 1)): J_kl = -c int int sum_i d_xi_i Psi_k F'(w)
 * Psi_l with c = dt / h on every axis. method: RIDG_ASM_QUADRATURE (every entry by tensor Gauss
 * quadrature), RIDG_ASM_QQF (F'(w) projected on the space-time basis by quadrature, then contracted with
 * the exact triple products), RIDG_ASM_PERTURBATION (central differences of the residual volume term,
 * eps = 1e-3, one pair of residual evaluations per unknown). w: device array [n_elements][theta_T]
 * (coefficients of each element's iterate); jac: device array [n_elements][theta_T][theta_T] (row = test
 * function k). Queued on hip_stream. The first call for a (device, dim, order) builds the point and
 * triple-product tables on the host and keeps a device copy until the process ends. Used to compare
 * the three assembly costs; the Burgers solver itself assembles quasi-quadrature-free. */
#define RIDG_ASM_QUADRATURE 0
#define RIDG_ASM_QQF 1
#define RIDG_ASM_PERTURBATION 2
int ridg_assemble_jacobian(int32_t method, int32_t dim, int32_t order, const double* w, int64_t n_elements,
                           double dt_over_h, double* jac, void* hip_stream);

/* Wait for all queued work of the handle. */
int ridg_synchronize(ridg_t* h);

/* Release the handle (not the workspace). NULL is accepted. */
int ridg_destroy(ridg_t* h);

/* Host-only von Neumann analysis (Sec. 1 and Sec. 6.1: the stable CFL of RIDG does not shrink with
 * the order): the largest modulus of an eigenvalue of the constant-velocity step's amplification
 * matrix I + sum_o K_o e^{i kappa.o} (K_o the composed prediction and correction taps) over a grid
 * of nk points per axis (2 <= nk <= 4096; at most 2^22 grid points). RIDG_E_INVAL for a
 * non-constant velocity. */
int ridg_host_spectral_radius(const ridg_problem* problem, double dt, int32_t nk, double* radius);

/* Host-only inspection of the FP64 precompute (no device needed).
 * Dense region matrix of element e for step dt as assembled by the library
 * (QQF): size (3^d theta_T)^2, row-major, blocks ordered by region offset
 * (o_1..o_d) in {-1,0,1}^d lexicographically with o_1 slowest, rows = test
 * functions. count must equal the number of entries. */
int ridg_host_region_matrix(const ridg_problem* problem, int64_t element, double dt, double* a,
                            size_t count);

/* Constant velocity: the prefactored prediction operator G (theta_T x 3^d
 * theta, row-major, column blocks in the region-offset order above) such
 * that W_e = G [Q_{e+o}]_o. */
int ridg_host_prediction_operator(const ridg_problem* problem, double dt, double* g, size_t count);

const char* ridg_error_string(int code);
/* Message of the last error on the calling thread (empty if none). */
const char* ridg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RIDG_H_ */
