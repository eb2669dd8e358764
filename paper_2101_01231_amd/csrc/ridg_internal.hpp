// Internal declarations of libridg: host FP64 precompute and device launchers.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ridg.h"

namespace ridg {

constexpr int kMaxDim = 3;
constexpr int kMaxOrder = 5;
constexpr int kMaxOrderQ1 = 12;  // tensor basis in 1D (composite stencil only)
constexpr int kMaxBlocks = 27;  // 3^3 region elements
constexpr uint8_t kOwn = 0xFF;  // plan face source: own trace (region boundary or outflow face)

// ---------------------------------------------------------------- basis
struct Basis {
  int d = 0, M = 0, family = RIDG_BASIS_P;
  int theta = 0, theta_t = 0;
  std::vector<std::array<int, 4>> sidx;  // spatial exponents (a_1..a_d)
  std::vector<std::array<int, 4>> tidx;  // space-time exponents (b_t, b_1..b_d)
};
Basis make_basis(int d, int M, int family = RIDG_BASIS_P);

// Exact 1D integrals of psi_m = sqrt(2m+1) P_m on [-1, 1].
double leg_t3(int a, int b, int c);  // int psi_a psi_b psi_c
double leg_d3(int a, int b, int c);  // int psi_a' psi_b psi_c
double leg_dm(int a, int b);         // int psi_a' psi_b
double leg_end(int m, int s);        // psi_m(s), s = +-1

// Reference tensors of the QQF assembly. The velocity component nu_i is
// projected on the p-modes {1, psi_1(xi_1), .., psi_1(xi_d)} (index p = 0,
// 1+j); tensors carry the face sign s where a face is involved.
struct RefTensors {
  int d = 0, nt = 0, ns = 0, np = 0;
  std::vector<double> Tt;   // [k][l]            time term
  std::vector<double> Cc;   // [k][l] (nt x ns)  causal source
  std::vector<double> Bv;   // [i][p][k][l]      int d_i Psi_k Psi_p Psi_l
  std::vector<double> Fo;   // [i][s][p][k][l]   s int Psi_k|s Psi_p Psi_l|s
  std::vector<double> Fn;   // [i][s][p][k][l]   s int Psi_k|s Psi_p Psi_l|-s
  std::vector<double> Cv;   // [i][p][k][l]      int d_i Phi_k Psi_p Psi_l (ns x nt)
  std::vector<double> CFo;  // [i][s][p][k][l]   s int Phi_k|s Psi_p Psi_l|s
  std::vector<double> CFn;  // [i][s][p][k][l]   s int Phi_k|s Psi_p Psi_l|-s
  std::vector<double> Cown; // [i][p][bits][k][l] Cv - CFo of the faces in bits (bit 0: s = -1, bit 1: s = +1)
  size_t bv(int i, int p) const { return ((size_t)i * np + p) * nt * nt; }
  size_t f(int i, int s, int p) const { return (((size_t)i * 2 + (s > 0)) * np + p) * nt * nt; }
  size_t cv(int i, int p) const { return ((size_t)i * np + p) * ns * nt; }
  size_t cf(int i, int s, int p) const { return (((size_t)i * 2 + (s > 0)) * np + p) * ns * nt; }
  size_t cown(int i, int p, int bits) const { return (((size_t)i * np + p) * 4 + bits) * ns * nt; }
};
RefTensors make_tensors(const Basis& b);

// ---------------------------------------------------------------- velocity
// v_i(x) = a_i + sum_j g_ij x_j with g_ii = 0 (divergence free, independent of x_i)
struct Affine {
  double a[3] = {0, 0, 0};
  double g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
};

struct Problem {
  int d = 0;
  int n[3] = {1, 1, 1};
  int M = 0;
  int flux = 0;
  Affine vel;
  double L[3] = {1, 1, 1};  // box side lengths
  double h[3] = {1, 1, 1};
  int precision = 0;
  int refine = 0;
  int solver = 0;  // resolved
  int newton_max = 0;  // RIDG_FLUX_BURGERS: Newton iterations per region at most
  int basis = RIDG_BASIS_P;
  int64_t nel = 0;
};

// Record msg as the calling thread's ridg_last_error() and return code.
int set_last_error(int code, const std::string& msg);

// Validate and resolve a public problem description. Returns RIDG_OK or an error (msg set).
int resolve_problem(const ridg_problem* p, Problem* out, std::string* msg);

// nu_i(xi) = c0[i] + sum_j c[i][j] xi_j on element idx for step dt.
void nu_coeffs(const Problem& P, const int idx[3], double dt, double c0[3], double c[3][3]);

// Upwind side of face (i, s) of element idx: 0 = own trace, 1 = neighbour trace,
// -1 = v.n changes sign inside the face.
int face_side(const Problem& P, const int idx[3], int i, int s);

// ---------------------------------------------------------------- plans
struct PlanBlock {
  int8_t off[3];
  int8_t pad0;
  uint8_t src[6];  // [2 i + (s > 0)]: kOwn or the plan position of the upwind source block
  uint8_t pad1[6];
};
static_assert(sizeof(PlanBlock) == 16, "plan block layout");

struct PlanRec {
  int32_t nb;
  int32_t pad[3];
  PlanBlock blk[kMaxBlocks];
};

struct RegionPlans {
  std::vector<PlanRec> plans;        // distinct acyclic plans
  std::vector<int32_t> elem_plan;    // plan id per element, -1 = centre on a dependency cycle
  std::vector<int32_t> tear_elems;   // cyclic regions solved by tearing one block (plan per element)
  std::vector<PlanRec> tear_plans;   // pad[0] = 1 (tear count), pad[1] = plan position of the centre
  std::vector<int32_t> dense_elems;  // remaining cyclic regions: dense LU of the whole region
};

// Offsets of the region blocks, lexicographic with o_1 slowest.
std::vector<std::array<int, 3>> region_offsets(int d);

void element_index(const Problem& P, int64_t e, int idx[3]);
int64_t element_linear(const Problem& P, const int idx[3]);  // periodic wrap

RegionPlans build_plans(const Problem& P);
// Plan of one element (false if its centre lies on a cycle).
bool element_plan(const Problem& P, int64_t e, PlanRec* out);
// Cyclic region: a plan whose block 0 is a tear block breaking every cycle among the centre's
// ancestors, the other ancestors following in elimination order (false if no single block does).
bool element_tear_plan(const Problem& P, int64_t e, PlanRec* out);

// Host FP64 assembly of the region matrix over the given region blocks (offsets), rows = tests.
// Interior faces between listed blocks are upwind; faces to unlisted blocks use the own trace
// when the block is on the 3^d region boundary, and are upwind couplings dropped otherwise (only
// used with ancestor-closed block sets, where such couplings do not exist).
void assemble_region(const Problem& P, const RefTensors& T, int64_t e, double dt,
                     const std::vector<std::array<int, 3>>& offs, std::vector<double>* A);

// Dense LU with partial pivoting (row-major n x n, in place); returns false on a zero pivot.
bool lu_factor(int n, double* a, int* piv);
void lu_solve(int n, const double* lu, const int* piv, double* b, int nrhs);  // b: n x nrhs row-major

// Constant velocity: taps (ancestor offsets) and G_r blocks (nt x ns each) of W_e = sum_r G_r Q_{e+r}.
struct Prefactored {
  std::vector<std::array<int, 3>> offs;
  std::vector<double> G;  // [tap][k][l]
};
int build_prefactored(const Problem& P, const RefTensors& T, double dt, Prefactored* out, std::string* msg);

// Constant velocity operators in tap form: out_e (+)= sum_t A_t in_{e + off_t}, A_t rows x cols.
struct TapOperator {
  std::vector<std::array<int, 3>> offs;
  std::vector<double> A;  // [tap][row][col]
  int rows = 0, cols = 0;
};
// Correction (Sec. 2.3) for constant velocity: Q'_e = Q_e + sum_t D_t W_{e + off_t} (own + inflow faces).
void build_correction_taps(const Problem& P, const RefTensors& T, double dt, TapOperator* out);
// Prediction and correction composed: Q'_e = Q_e + sum_o K_o Q_{e+o}, K_o = sum_{t+s=o} D_t G_s.
void build_composite(const Problem& P, const Prefactored& G, const TapOperator& Dc, TapOperator* out);
constexpr int kMaxTapUpdate = 125;  // composite offsets in {-2..2}^3
// Von Neumann analysis of the constant-velocity step Q' = Q + sum_o K_o Q_{.+o}: the largest
// modulus of an eigenvalue of I + sum_o K_o e^{i kappa.o} over a grid of nk points per axis.
double spectral_radius(const TapOperator& K, int d, int nk);
// The same for the problem's composed step at dt (grid: 256 points in 1D, 48^2 in 2D, 12^3 in 3D).
int von_neumann_radius(const Problem& P, const RefTensors& T, double dt, double* rho, std::string* msg);
constexpr double kUnstableRadius = 1.0 + 1e-10;
// A operator [tap][rows][cols] rearranged as MFMA A fragments: [row tile][tap][chunk][lane] holding
// A_t[16 tile + lane % 16][4 chunk + lane / 16], zero outside rows x cols (16x16x4 layout).
std::vector<double> mfma_fragments(const double* A, int ntaps, int rows, int cols);
inline size_t mfma_fragment_doubles(int ntaps, int rows, int cols) {
  return (size_t)((rows + 15) / 16) * ntaps * ((cols + 3) / 4) * 64;
}

// ---------------------------------------------------------------- device side
struct DevTensors {  // device copies (FP64), offsets into one buffer
  const double* Tt;
  const double* Cc;
  const double* Bv;
  const double* Fo;
  const double* Fn;
  const double* Cv;
  const double* CFo;
  const double* CFn;
  const double* Cown;
};

// Precombined region-block tensors of the upwind-plan kernel. For an affine velocity the
// transverse-slope modes V_{i,1+j} are the same on every element, so each diagonal block is
//   A_rr = A0[mask] + sum_i V_{i,0}(element) K_i[mask_i]
// with mask = sum_i own_i << 2i, own_i = (own trace on face s=-1) | (own trace on s=+1) << 1.
struct PlanTables {
  const double* A0;       // [mask][k][l]  Tt + sum_{i,j} V_{i,1+j} (-Bv[i][1+j] + sum_own Fo[i][s][1+j])   (dt)
  const double* K;        // [i][mask_i][k][l]  -Bv[i][0] + sum_own Fo[i][s][0]
  const double* Fn0;      // [i][sd][k][l]  Fn[i][s][0]
  const double* FnC;      // [i][sd][k][l]  sum_j V_{i,1+j} Fn[i][s][1+j]                                 (dt)
  const int32_t* cc_idx;  // [k] the spatial mode coupled to Psi_k by the causal source
  const double* cc_val;   // [k] its coefficient
};

struct HostPlanTables {
  std::vector<double> A0, K, Fn0, FnC, cc_val;
  std::vector<int32_t> cc_idx;
};
HostPlanTables build_plan_tables(const Problem& P, const RefTensors& T, double dt);
int plan_max_blocks(int d);

struct DevGeom {
  int d, n0, n1, n2;
  double h0, h1, h2;
  double a[3];
  double g[3][3];
};

// Serving: per-problem descriptors passed by value to the shared launches (k_batch.hip).
constexpr int kBatchTaps = 8;  // constant velocity: the upwind cone has at most 2^d taps
constexpr int kBatchMax = 16;  // problems per launch (kernel-argument budget)
struct BatchDesc {
  const double* Qin;
  double* Qout;
  double* W;
  const double* G;
  const double* Dc;  // correction taps (theta x theta_T each)
  int64_t block_begin;  // first workgroup of this problem in the launch grid
  int64_t nel;
  double h[3];
  double v[3];
  double dt;
  int32_t n[3];
  int32_t ntaps;
  int32_t ndtaps;
  int8_t taps[kBatchTaps][3];
  int8_t dtaps[7][3];
  int8_t pad[7];
};
struct BatchArgs {
  BatchDesc d[kBatchMax];
  int32_t count;
  int32_t pad;
};
int launch_batch_step(int d, int M, const BatchArgs& args, const DevTensors& t, void* stream);

// Batched MFMA tap products (prediction or correction of several constant-velocity problems of one
// (dimension, order) family in one launch); workgroups [group_begin, next group_begin) serve a problem.
struct BatchMfmaDesc {
  const double* in;
  const double* base;  // nullptr: out = product
  double* out;
  const double* frag;  // MFMA fragments of the operator (mfma_fragments)
  int64_t group_begin;
  int64_t tiles_per_group;
  int32_t n[3];
  int32_t ntaps;
  int8_t taps[kBatchTaps][3];
};
struct BatchMfmaArgs {
  BatchMfmaDesc d[kBatchMax];
  int32_t count;
  int32_t pad;
};
struct BatchMfmaTaps {
  int8_t off[kBatchTaps][3];
};
int mfma_tiles_per_group(int64_t nel, size_t lds_bytes);  // tiles a workgroup sweeps (fragments staged: lds_bytes)
int launch_batch_mfma(int d, int M, int kind, const BatchMfmaArgs& args, int64_t groups, void* stream);

// Launchers (defined in the k_*.hip units). All return a hipError_t as int.
int launch_aos_to_soa(const double* src, double* dst, int64_t nel, int nmodes, void* stream);
int launch_soa_to_aos(const double* src, double* dst, int64_t nel, int nmodes, void* stream);
int launch_predict_prefactored(int d, int M, const DevGeom& g, const double* Q, double* W,
                               const double* G, const int32_t* taps, int ntaps, void* stream);
// kind 0: correction taps (W -> Q' = Q + ...), kind 1: composite taps (Q -> Q' = Q + ...)
int launch_tap_update(int d, int M, int kind, const DevGeom& g, const double* in, const double* base, double* out,
                      const double* A, const int32_t* taps, int ntaps, void* stream);
// The composite stencil in 3D marched along z with a ring of three state planes in LDS (k_stencil3d.hip):
// theta 4 or 10 (orders 2-3), n0 and n1 multiples of 16, n2 a multiple of 8 or at most 64.
struct ZMarch {
  int8_t lo[3], hi[3];  // tap offset range per axis (span <= 2)
  int32_t tz;           // planes per workgroup
};
bool zmarch_supported(int d, int ns, int n0, int n1, int n2);
int launch_tap_zmarch(int ns, const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps,
                      int ntaps, void* stream);
// The composite stencil for ns spatial modes (the tensor basis: ns = M in 1D up to 12, M^2 in 2D up to 25).
int launch_tap_composite_ns(int d, int ns, const DevGeom& g, const double* in, double* out, const double* A,
                            const int32_t* taps, int ntaps, void* stream);
// The same tap operators on FP64 MFMA; frag = mfma_fragments(...) of the operator (device copy).
constexpr int kMfmaPredict = 0, kMfmaCorrect = 1, kMfmaComposite = 2;
constexpr size_t kMfmaMaxLds = 160 * 1024;  // fragments up to this size are staged in LDS
int launch_tap_mfma(int d, int M, int kind, const DevGeom& g, const double* in, const double* base, double* out,
                    const double* frag, const int32_t* taps, int ntaps, void* stream);
// layout: 0 = packed theta_T-lane segments, 1 = power-of-two segments (DPP reductions)
int launch_predict_plans(int d, int M, int layout, int precision, int refine, const DevGeom& g, double dt,
                         const double* Q, double* W, const PlanTables& t, const PlanRec* plans,
                         const int32_t* items, const int32_t* item_plan, int64_t n_items, void* stream);
// plan-kernel segment layouts: 0 packed, 1 padded to a power of two, 2 two regions per packed
// segment, 3 two rows per lane, 4 several rows per lane in power-of-two (DPP) segments, 5 the
// layout-4 geometry with static pivots (row c pivots column c)
constexpr int kLayouts = 6;
constexpr int kStaticPivotLayout = 5;
int items_per_wave(int d, int M, int layout);
// the FP64-only layouts (separate translation units)
int launch_plans2(int d, int M, const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t,
                  const PlanRec* plans, const int32_t* items, const int32_t* item_plan, int64_t n_items, void* stream);
int launch_plans_2rows(int d, int M, const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t,
                       const PlanRec* plans, const int32_t* items, const int32_t* item_plan, int64_t n_items,
                       void* stream);
int launch_plans_dpp(int d, int M, const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t,
                     const PlanRec* plans, const int32_t* items, const int32_t* item_plan, int64_t n_items,
                     void* stream);  // work-list padding multiple (regions a wavefront takes at once)
// static pivots (layout 5): FP64 or RIDG_FP32_REFINE with `refine` FP64-residual sweeps
int launch_plans_sp(int d, int M, int precision, int refine, const DevGeom& g, double dt, const double* Q, double* W,
                    const PlanTables& t, const PlanRec* plans, const int32_t* items, const int32_t* item_plan,
                    int64_t n_items, void* stream);
// Largest growth factor max|U| / max|A| of elimination without row exchanges over the diagonal
// region blocks A0[mask] + sum_i V_i K_i[mask_i] of the tables, for V on a grid spanning the
// problem's range of V_i0 = v_i(element centre) dt / h_i (inf where a pivot vanishes).
double static_pivot_growth(const Problem& P, const HostPlanTables& H, int nt, double dt);
constexpr double kStaticPivotMaxGrowth = 64.0;
// Fused constant-velocity 3D step on bricks (k_brick.hip): predictions of a brick and its upwind halo
// on the matrix cores (FP64, or FP32 operands and accumulation when f32), FP64 correction.
struct BrickTaps {
  int8_t g[8][3];  // prediction taps (upwind cone)
  int8_t d[4][3];  // correction taps (own element, inflow faces)
  int32_t ng, nd;
  int8_t wlo[3], whi[3];  // prediction region: the brick extended by [wlo, whi] per axis
  int8_t qlo[3], qhi[3];  // state region: the prediction region extended by the prediction taps
};
bool brick_supported(int d, int M, const int n[3], bool f32);
// frag: mfma_fragments of G (one row tile; doubles, or the same values as floats when f32)
int launch_brick_step(int M, bool f32, const DevGeom& g, const double* Q, double* Qout, const void* frag,
                      const double* Dc, const BrickTaps& tp, void* stream);

// Whole run of n_steps on one workgroup (mesh state resident in LDS), constant velocity;
// returns hipErrorInvalidValue when the mesh does not fit.
int fused_fits(int d, int M, int64_t nel);
int launch_fused_prefactored(int d, int M, const DevGeom& g, double dt, const double* Qin, double* Qout,
                             const double* G, const int32_t* taps, int ntaps, const DevTensors& t, int n_steps,
                             void* stream);
int launch_predict_tear(int d, int M, const DevGeom& g, double dt, const double* Q, double* W,
                        const PlanTables& t, const PlanRec* plans, const int32_t* elems, int64_t n_elems,
                        void* stream);
int launch_predict_dense(int d, int M, const DevGeom& g, double dt, const double* Q, double* W,
                         const DevTensors& t, const int32_t* elems, int64_t n_elems, double* scratch,
                         int64_t scratch_elems, void* stream);
int launch_correct(int d, int M, int flux, const DevGeom& g, double dt, const double* Q, const double* W,
                   double* Qout, const DevTensors& t, void* stream);
int launch_check_finite(const double* x, int64_t n, int32_t* flag, void* stream);

// ---------------------------------------------------------------- Burgers (Newton prediction)
// Orders the Newton path implements per dimension (region system of 3^d theta_T unknowns).
bool burgers_supported(int d, int M);
// Gauss-Legendre points per axis of the Burgers tables: exact for the products of a basis function
// with F(w) = w^2 / 2 or with F'(w) and a second basis function (per-axis degree 3M - 3).
constexpr int burgers_q(int M) { return (M + 1) > (3 * M - 1) / 2 ? (M + 1) : (3 * M - 1) / 2; }
// Host tables (FP64) of the Newton prediction and the nonlinear correction; point sets are the tensor
// Gauss rules on the space-time element (volume, q^(d+1) points) and on its faces (q^d points
// (tau, xi_perp); face f = 2 i + (s > 0) lies at xi_i = s).
struct BurgersHost {
  int q = 0, nq = 0, nqf = 0;
  std::vector<double> psiv;    // [l][pt]      Psi_l at the volume points
  std::vector<double> dpsivw;  // [i][k][pt]   w_pt d_xi_i Psi_k (residual volume term)
  std::vector<double> projw;   // [p][pt]      w_pt Psi_p / 2^(d+1) (projection onto Psi, eq. Jacproj)
  std::vector<double> dphivw;  // [i][k][pt]   w_pt d_xi_i Phi_k (correction volume term)
  std::vector<double> psif;    // [f][l][pf]   Psi_l at the points of face f
  std::vector<double> psifw;   // [f][k][pf]   w_pf Psi_k on face f
  std::vector<double> phifw;   // [f][k][pf]   w_pf Phi_k on face f
  std::vector<int32_t> bptr;   // [i][k][l] -> first entry of (k, l) in bp / bval (size d nt^2 + 1)
  std::vector<int32_t> bp;     // p of each non-zero beta^i_{k l p} = int d_xi_i Psi_k Psi_p Psi_l
  std::vector<double> bval;
  std::vector<int32_t> lift;   // [j] space-time index of spatial mode j held constant in time
};
int build_burgers_tables(const Problem& P, const Basis& B, BurgersHost* out, std::string* msg);
// Device view of the same tables (pointers into the workspace).
struct BurgersDev {
  const double *Tt, *Cc;
  const double *psiv, *dpsivw, *projw, *dphivw, *psif, *psifw, *phifw, *bval;
  const int32_t *bptr, *bp, *lift;
};
// Newton prediction of every element (one workgroup per region, the region Jacobian in LDS); stats:
// [0] max iterations, [1] failures, [2..3] total iterations (int64), [4..5] region solves (int64).
int launch_burgers_predict(int d, int M, const DevGeom& g, double dt, const double* Q, double* W,
                           const BurgersDev& t, int64_t nel, int max_iter, int32_t* stats, void* stream);
int launch_burgers_correct(int d, int M, const DevGeom& g, double dt, const double* Q, const double* W,
                           double* Qout, const BurgersDev& t, void* stream);

// ---------------------------------------------------------------- Jacobian assembly comparison (Sec. 3)
// Volume block J_kl = -c int int sum_i d_xi_i Psi_k F'(w) Psi_l of the Burgers flux (F'(w) = w) on
// the space-time element, c = dt / h on every axis, by quadrature, by quasi-quadrature-free projection
// (F'(w) projected on Psi, then the exact triple products summed over the directions), or by central
// differences of the residual volume term, one column per unknown.
struct AsmHost {
  int nt = 0, q = 0, nq = 0;
  std::vector<double> psiv;   // [l][pt] Psi_l at the volume points
  std::vector<double> projw;  // [p][pt] w_pt Psi_p / 2^(d+1)
  std::vector<double> dsum;   // [k][pt] w_pt sum_i d_xi_i Psi_k
  std::vector<int32_t> rptr;  // [k][l] -> first entry in bp / bval (size nt^2 + 1)
  std::vector<int32_t> bp;    // p of each non-zero sum_i beta^i_{k l p}
  std::vector<double> bval;
};
int build_assembly_tables(int d, int M, AsmHost* out, std::string* msg);
struct AsmDev {
  int nt, nq;
  const double *psiv, *projw, *dsum, *bval;
  const int32_t *rptr, *bp;
};
constexpr int kAsmQuadrature = 0, kAsmQqf = 1, kAsmPerturbation = 2;
int launch_assembly(int method, const AsmDev& t, int64_t n_elements, const double* W, double c, double* J,
                    void* stream);

}  // namespace ridg
