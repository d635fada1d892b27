// Internal launcher interfaces between the gfx950 kernels and the host code.
#pragma once
#include "common.h"

namespace sb {

enum Dtype {
  DT_F64 = SB_DTYPE_F64,
  DT_F32 = SB_DTYPE_F32,
  DT_BF16 = SB_DTYPE_BF16,
  DT_F32S = SB_DTYPE_F32_SPLIT  // FP32 data, contraction as three BF16 products
};

// Device-side view of a likelihood (all pointers are device pointers).
struct Model {
  int family = 0, norm = 0, d = 0, K = 0;
  const double *mu64 = nullptr;   // [K][d]
  const double *P64 = nullptr;    // [K][d][d]
  const double *beta = nullptr;   // [K]
  const float *mu32 = nullptr;    // [K][d] (FP32 / BF16 paths)
  const void *Plp = nullptr;      // [K][d][d] FP32 or BF16 copy
  const bf16_t *Phi = nullptr;    // [K][d][d] bf16(P) (BF16 and split contractions)
  const bf16_t *Plo = nullptr;    // [K][d][d] bf16(P - hi) (split contraction)
  double nu = 0.0, c = 0.0;       // Student-t dof, additive constant
};

// ------------------------------------------------------------------ batches
// A batch of n independent problems laid out side by side in packed arrays.
// Problem p's vectors have length dp = d rounded up to a multiple of 8; the
// padding of every vector, mean and precision row is exactly zero and stays
// zero through the GEMM (zero P rows/columns) and the optimiser (zero
// gradient there).  A single problem is a batch of one.
struct BatchProb {
  int d = 0, dp = 0, K = 0, family = 0, norm = 0, n_pts = 0;
  double nu = 0.0, c = 0.0;
  int64_t P_off = 0;     // packed P: component k of p at P_off + k*dp*dp
  int64_t mu_off = 0;    // packed mu: P's component k at mu_off + k*dp
  int64_t beta_off = 0;  // packed beta / log det P: beta_off + k
  int64_t box_off = 0;   // packed lo/hi: box_off + i, i < dp (padding unused)
  int64_t s0 = 0, B = 0, voff0 = 0;           // starts: global index, count, vector offset
  int64_t r0 = 0, R = 0, roff0 = 0, pt0 = 0;  // rays: global index, count, endpoint offset, first point row
  uint64_t seed = 0;                          // Philox key of this problem's rays
  int32_t index = 0;                          // problem number (Philox counter word 3)
};

// Device tables of a batch (all device pointers).
struct BatchDev {
  int n = 0;                          // problems
  const BatchProb *probs = nullptr;   // [n]
  int64_t Btot = 0, Ltot = 0;         // starts, sum of B_p * dp_p
  int64_t Rtot = 0, RLtot = 0, NPtot = 0;  // rays, sum R_p * dp_p, sum R_p * n_pts_p
  int dp_max = 0, K_max = 0;
  const double *P64 = nullptr, *mu64 = nullptr, *beta = nullptr, *lo = nullptr, *hi = nullptr;
  const float *P32 = nullptr, *mu32 = nullptr;
  const bf16_t *Pbf = nullptr;
};

// A row segment of a grouped GEMM: rows [row0, row0 + rows) all belong to
// problem `prob`; their Y rows (K*dp each) start at element yoff and their
// q-partial rows (K*ntn each, ntn = ceil(dp / bn)) at element qoff.
struct GSeg {
  int32_t prob = 0, rows = 0;
  int64_t row0 = 0, yoff = 0, qoff = 0;
};

// Grouped GEMM view: each M-tile belongs to one segment (static table).
struct GroupView {
  const BatchProb *probs = nullptr;
  const GSeg *segs = nullptr;
  int nseg = 0;
  const int32_t *tile_seg = nullptr;   // [grid.x] segment of the M-tile
  const int32_t *tile_idx = nullptr;   // [grid.x] tile index within the segment
  const int32_t *counts = nullptr;     // [nseg] active rows per segment (nullable: segs[].rows)
  int kind = 0;                        // 0: rows of X (rowoff), 1: ray points of the problem
  const int64_t *rowoff = nullptr;     // kind 0: global row -> element offset of its X row
  const void *mu = nullptr, *P = nullptr;  // packed mu / P in the GEMM's input / operand types
};

// Source of the A operand (the points) of the quadratic-form GEMM.
struct ASrc {
  int kind = 0;                   // 0: rows of X; 1: ray points p + t (q - p)
  const void *X = nullptr;        // kind 0: [rows][ldx], double (F64) or float (F32/BF16)
  int64_t ldx = 0;
  const int32_t *rowmap = nullptr;// kind 0: GEMM row r reads X row rowmap[r] (nullable)
  int64_t rows = 0;               // kind 0: rows of X (0: the GEMM's row count)
  const void *P0 = nullptr, *P1 = nullptr;  // kind 1: [R][d] endpoints, same type as X
  int n_pts = 1;
  // kind 1: point jj of a ray at t = t0 + jj dt when dt > 0 (BF16 kernel
  // only; three nodes of the ray-quadratic scores), else (jj + 1/2) / n_pts
  float t0 = 0.f, dt = 0.f;
  bool zero_mu = false;           // A = X instead of X - mu_k
};

// Outputs of the GEMM: Y = (X - mu_k) P_k^T per component (optional) and
// per-tile partial quadratic forms sum_n delta_n Y_n.
struct QuadOut {
  void *Y = nullptr;              // [M][ldy] accumulation type, columns k*d + n
  int64_t ldy = 0;
  void *qpart = nullptr;          // [M][K][ntn]
  int ntn = 0;                    // set by the launcher (n-tiles per component)
  // BF16 kernels only: q partials as sums of squares of (X - mu_k) U_k^T with
  // the model's B operand U_k = L_k^T (no Y); Y rows through ymap and its
  // column block at ycol
  bool sumsq = false;
  const int32_t *ymap = nullptr;
  int64_t ycol = 0;
  // grouped by component: gcnt[k] rows of component k listed at
  // a.rowmap + k * gcap and ymap + k * gcap (M = list capacity); qpart is
  // then indexed by the Y row
  const int32_t *gcnt = nullptr;
  int64_t gcap = 0;
  bool yneg = false;  // store -Y (a Gaussian's gradient); q still uses Y
  // BF16 kernels, grouped: gdst + k * gcap lists beside ymap the gradient
  // row of each listed row that has no other listed component (its only
  // responsibility is exactly 1), else -1; such a row takes -Y in that row
  // of gdir [*][ldg] instead of its Y block (q still uses Y)
  const int32_t *gdst = nullptr;
  void *gdir = nullptr;
  int64_t ldg = 0;
};

// Tile shape used for a GEMM call; chosen by the autotuner.
struct TileCfg {
  int bm = 128, bn = 128;
  int bk = 32;      // k-tile: BF16 kernels 32 or 64; FP32 16 or 32; FP64 16 or 32 (32 at
                    // 32x64, 64x64, 128x64, 64x128 only)
  int stages = 1;  // BF16 kernels: LDS stages (2 = ping-pong, square tiles, k-tile 32)
};

int quad_gemm_ntn(int dtype, int d, TileCfg t);
// "BMxBN[xBK[xSTAGES]]" (an environment override) into *t; false if
// e is null or malformed (t untouched).
bool parse_tile(const char *e, TileCfg *t);
// BF16 matrix-core contraction (d a multiple of 8): nprod 1 = BF16 operands,
// 3 = split FP32 operands (hi*hi + hi*lo + lo*hi); Y and qpart in FP32.
bool quad_gemm_bf16_ok(int d);
// t selects the variant: t.bm rows per tile (128 / 256), t.bn the k-tile (32 / 64).
int launch_quad_gemm_bf16(int nprod, const Model &m, const ASrc &a, int64_t M,
                          const int32_t *count, QuadOut &o, hipStream_t s, TileCfg t);
// hi = bf16(fp32(x)), lo = bf16(x - hi) (lo nullable) for n values.
int launch_split_bf16(int64_t n, const double *x, bf16_t *hi, bf16_t *lo, hipStream_t s);
// hi/lo split of U_k = L_k^T from K lower Cholesky factors [K][d][d].
int launch_split_upper(int K, int d, const double *L, bf16_t *hi, bf16_t *lo, hipStream_t s);
int launch_quad_gemm(int dtype, const Model &m, const ASrc &a, int64_t M, const int32_t *count,
                     QuadOut &o, TileCfg t, hipStream_t s);

// Row epilogue: l (and gradient, responsibilities) from qpart / Y.
struct FinishArgs {
  int64_t M = 0;
  const int32_t *count = nullptr;   // device row count (nullable -> M)
  const int32_t *outmap = nullptr;  // row -> output row (nullable)
  const void *qpart = nullptr;
  int ntn = 0;
  const void *Y = nullptr;
  int64_t ldy = 0;
  void *logl = nullptr;             // [*] acc type
  void *grad = nullptr;             // [*][ldg] acc type (nullable)
  int64_t ldg = 0;
  void *aux = nullptr;              // [M][K]: responsibilities (mixture) / q (Student-t)
  bool logl_f64 = false;            // l output is FP64 whatever the operand type
  // mixture with l and FP32 responsibilities [M][K] already computed (by the
  // mixture-rows pass): the epilogue forms the gradient only
  const void *resp = nullptr;
  // with resp: rows whose component mask has a single bit had their gradient
  // written by the contraction (QuadOut::gdst) and are skipped
  const uint32_t *skip1 = nullptr;
};
int launch_finish(int dtype, const Model &m, const FinishArgs &f, hipStream_t s);
// FP64 logL + gradient of rows of X in one launch (contraction and row
// epilogue fused; small dimensions: d <= 128, K * round_up(d, 32) <= 384, Gaussian
// mixture or single-component Student-t).  Same outputs as launch_quad_gemm +
// launch_finish with FP64 l (aux: responsibilities / q), no Y.
// C[b][n] = c0[n] + sum_k A[b][k] Bp[k sk + n sn] in FP64 on the matrix
// cores (c0 nullable; b < B, n < N, k < Kd).
int launch_small_gemm_f64(int64_t B, int N, int Kd, const double *A, int64_t lda, const double *Bp,
                          int64_t sk, int64_t sn, const double *c0, double *C, int64_t ldc,
                          hipStream_t s);
// Bounds of the reduced box: per column i < r of V [d][ldv] the interval of t
// with theta* + t V[:, i] inside [lo, hi].
int launch_reduced_bounds(int d, const double *th, const double *V, int64_t ldv, int r,
                          const double *lo, const double *hi, double *plo, double *phi,
                          hipStream_t s);
bool fused_logl_grad_ok(const Model &m, const ASrc &a);
int launch_fused_logl_grad(const Model &m, const ASrc &a, int64_t M, const int32_t *count,
                           const int32_t *outmap, double *logl, double *grad, int64_t ldg,
                           double *aux, hipStream_t s);
// Gaussian-mixture rows from FP32 q partials: l, FP32 responsibilities, and
// per component the rows whose responsibility is not zero.
struct MixRowsArgs {
  int64_t M = 0;
  const int32_t *count = nullptr;   // device row count (nullable -> M)
  const float *qpart = nullptr;     // [M][K][ntn]
  int ntn = 0;
  const int32_t *rowmap = nullptr;  // operand row of each row (nullable: the row)
  const int32_t *outmap = nullptr;  // l output row (nullable: the row)
  void *logl = nullptr;
  bool logl_f64 = false;
  float *resp = nullptr;            // [M][K]
  int32_t *cnt = nullptr, *rows = nullptr, *xrows = nullptr;  // [K], [K][cap], [K][cap]
  int64_t cap = 0;
};
int launch_mixture_rows(const Model &m, const MixRowsArgs &a, hipStream_t s);

// Screened mixture rows (FP32 rows of X).  Each operand row carries its last
// evaluated point x_ref with bounds lb_k <= sqrt(q_k(x_ref)) <= ub_k; at a new
// point x the bounds widen by sigma_k |x - x_ref| (sigma_k^2 >= the largest
// eigenvalue of P_k) and only the components they cannot rule out are listed
// for the contraction; every other one gets q partials (+inf, 0, ...) in
// qpart and keeps the widened bounds.  x becomes the new x_ref.  After the
// contraction the post pass forms l and the responsibilities (the epilogue's
// own function) and sets the listed components' bounds from their q_k.
struct ScreenArgs {
  int64_t M = 0;
  const int32_t *count = nullptr;   // device row count (nullable -> M)
  const float *X = nullptr;         // operand rows (FP32), row stride ldx
  int64_t ldx = 0;
  const int32_t *rowmap = nullptr;  // operand row of each row (nullable: the row)
  int64_t nstate = 0;               // operand rows with screening state
  const double *rho = nullptr;      // [K] max_i sum_j |P_k[i][j]| (>= the largest eigenvalue)
  float *xref = nullptr;            // [nstate][d] last evaluated points
  double *bnd = nullptr;            // [nstate][2K] lb_k then ub_k
  int32_t *hasref = nullptr;        // [nstate] 1: x_ref and bounds set, else none yet
  float *nrm = nullptr;             // [cap][K] |x - mu_k|^2 of the listed components
  float *qpart = nullptr;           // [M][K][ntn] q partials of the contraction
  int ntn = 0;
  uint32_t *mask = nullptr;         // [cap] components listed per row (bit k)
  int32_t *gdst = nullptr;  // [K][cap] (nullable): beside rows, the output row of a row
                            // listed for one component only, else -1
  int32_t *cnt = nullptr, *rows = nullptr, *xrows = nullptr;  // [K], [K][cap], [K][cap]
  int64_t cap = 0;
  // post pass: l (at outmap[row], FP64 or FP32) and r [M][K]
  void *logl = nullptr;
  const int32_t *outmap = nullptr;
  bool logl_f64 = false;
  float *resp = nullptr;
};
// screen + list passes (the screen zeroes cnt)
int launch_mixture_screen(const Model &m, const ScreenArgs &a, hipStream_t s);
int launch_mixture_post(const Model &m, const ScreenArgs &a, hipStream_t s);
// rho[k] = max_i sum_j |P_k[i][j]| (FP64 P [K][d][d]); rho is zeroed first.
int launch_row_abs_max(int K, int d, const double *P, double *rho, hipStream_t s);
// Tightens rho[k] (an upper bound of P_k's largest eigenvalue) to
// min(rho[k], tau_k (1 + 2^-20)) where tau_k = 1.25 theta_k, theta_k the
// Rayleigh quotient after 16 power steps, whenever the Cholesky factorisation
// of tau_k I - P_k succeeds (which certifies tau_k above every eigenvalue up
// to the factorisation's backward error).  work: 2 K d + K doubles; A: K d^2
// doubles of scratch; info: K ints.
int launch_lmax_bound(int K, int d, const double *P, double *rho, double *work, double *A,
                      int32_t *info, hipStream_t s);

struct HvpArgs {
  int64_t M = 0;
  const void *qpart = nullptr;
  int ntn = 0;
  const double *Y = nullptr, *Z = nullptr;
  int64_t ldy = 0;
  const double *V = nullptr;
  double *HV = nullptr;
};
int launch_hvp_finish(const Model &m, const HvpArgs &h, hipStream_t s);

// H[c] = -nabla^2 l from Y, aux (responsibilities or q) and grad (FP64).
int launch_hessian_assemble(const Model &m, int C, const double *Y, int64_t ldy,
                            const double *aux, const double *grad, double *H, hipStream_t s);

// Precision conversions and prep.
int launch_convert_model(const Model &m, float *P32, bf16_t *Pbf, float *mu32, hipStream_t s);
int launch_symmetry_check(const double *P, int K, int d, double *mx, int32_t *bad, hipStream_t s);
int launch_beta(const Model &m, const double *log_w, const double *logdetP, double *beta,
                hipStream_t s);

// Cholesky (FP64, batched), log det, solve.
int chol_batched(int C, int n, const double *A, double *L, int32_t *info, hipStream_t s);
int launch_logdet(int C, int n, const double *L, const int32_t *info, double *logdet,
                  hipStream_t s);
int launch_chol_solve(int C, int n, const double *L, const double *b, double *x,
                      const int32_t *info, hipStream_t s);

// Rays / discovery.
int launch_rays(int d, const double *lo, const double *hi, int R, uint64_t seed,
                uint32_t problem, double *P0, double *P1, float *P0f, float *P1f, hipStream_t s);
// Scores of R rays x n_pts sample points, t_j = (j + 1/2) / n_pts, from the
// FP32 q partials of three nodes per ray (t = 0, 1/2, 1; qpart rows 3 r + i):
// each q_k is a quadratic polynomial in t along a ray, so Lagrange
// interpolation of the node values gives it at every sample; then the
// family's l in FP64, written as FP32 l [R][n_pts].
int launch_ray_nodes_finish(const Model &m, int64_t R, int n_pts, int ntn, const float *qpart,
                            float *l, hipStream_t s);
// BF16 discovery scores by the ray-quadratic shortcut: the BF16 contraction at
// the three nodes of each ray (P0/P1 FP32 endpoints), then the interpolation.
// qpart holds >= 3 R K ceil(d/64) floats, l R n_pts floats; the tile is
// autotuned on these operands.  Needs quad_gemm_bf16_ok(d).
int discover_bf16_nodes(const Model &m, const float *P0, const float *P1, int R, int n_pts,
                        float *qpart, float *l, hipStream_t s);
// Preprocessing probe (precheck.hip): s [d], cls [d] (0 active, 1 flat,
// 2 soft nuisance) and the marginal log-evidence *logz (device); the host gets
// counts_host [4] = active, flat, soft, non-finite sensitivities.
size_t precheck_ws_bytes(int d, int K);
int run_precheck(const Model &m, const double *lo, const double *hi, double eps_flat,
                 double eps_soft, double *s, int32_t *cls, double *logz, int32_t *counts_host,
                 void *workspace, size_t ws_bytes, hipStream_t st);
// Eigendecomposition and dimensional reduction at modes (reduce.hip): C
// symmetric n x n matrices H; eigval [C][n] descending, V [C][n][n] (column i
// = eigenvector of eigval i), cls [C][n], marginal log-evidence logz [C]
// (device); deff_host [C] and *sweeps_host on the host.
size_t reduce_ws_bytes(int C, int n);
int run_eig_reduce(int C, int n, const double *H, const double *lo, const double *hi,
                   double eps_inform, double eps_nuis, double *eigval, double *V, int32_t *cls,
                   double *logz, int32_t *deff_host, int32_t *sweeps_host, void *workspace,
                   size_t ws_bytes, hipStream_t st);
int launch_ray_argmax(int R, int n_pts, int dtype, const void *l, double *best_l, int32_t *best_j,
                      hipStream_t s);
int launch_topn(int R, int n_starts, const double *best_l, int32_t *start_ray, hipStream_t s);
int launch_gather_starts(int d, int n_pts, int n_starts, const int32_t *start_ray,
                         const int32_t *best_j, const double *P0, const double *P1, double *X0,
                         hipStream_t s);

// Misc elementwise helpers.
int launch_cast_f64_f32(int64_t n, const double *a, float *b, hipStream_t s);
int launch_cast_f32_f64(int64_t n, const float *a, double *b, hipStream_t s);
int launch_fill_i32(int64_t n, int32_t v, int32_t *p, hipStream_t s);

// Batched L-BFGS (state machine over starts).
struct LbfgsBuffers {
  int dtype = DT_F64;
  bool hist_bf16 = false;  // FP32 starts: the history ring holds BF16 pairs (m <= kMaxHist)
  int64_t B = 0;
  int d = 0, m = 8;
  void *X = nullptr, *G = nullptr, *F = nullptr;  // [2][B][d], [2][B][d], [2][B] (F: FP64)
  void *Pd = nullptr;                             // [B][d]
  void *S = nullptr, *Yh = nullptr;               // [B][m][d]
  void *rho = nullptr, *yy = nullptr;             // [B][m]
  void *alpha = nullptr, *gtp = nullptr;          // [B]
  int32_t *cur = nullptr, *head = nullptr, *cnt = nullptr, *iters = nullptr, *ls = nullptr;
  int32_t *status = nullptr, *phase = nullptr, *rowid = nullptr, *active = nullptr;
  int32_t *idx = nullptr, *count = nullptr;       // compacted rows, [B] and [1]
  int64_t *evals = nullptr;                       // [1]
  // batches: per-start vector offset/length, total vector length, trial row
  // offsets (per start) and their compacted copy (per compacted row)
  const int64_t *voff = nullptr;
  const int32_t *vdim = nullptr;
  int64_t Ltot = 0;
  int64_t *rowoff = nullptr, *croff = nullptr;
  // batches: problem of each start, per-problem gradient tolerance and
  // iteration cap (nullable: the launch's scalars), per-problem evaluations
  const int32_t *sprob = nullptr;
  const double *ptol = nullptr;
  const int32_t *pmaxit = nullptr;
  int64_t *pevals = nullptr;
};

// Per-problem compaction of a batch's active starts: rows of problem p land
// at s0_p + i (i < counts[p]) in idx (F index) and croff (row offsets).
int launch_compact_group(const BatchDev &b, const LbfgsBuffers &lb, int32_t *counts,
                         hipStream_t s);
int launch_lbfgs_init_group(const LbfgsBuffers &b, const void *X0, hipStream_t s);
int launch_lbfgs_gather_group(const LbfgsBuffers &b, void *X, double *logl, int32_t *status,
                              hipStream_t s);

// Grouped GEMM and its epilogue over a batch.
struct FinishGroupArgs {
  const GSeg *segs = nullptr;        // row segments (as given to the GEMM)
  int nseg = 0;
  int64_t nrows = 0;                 // rows spanned by the segments
  const int32_t *rowseg = nullptr;   // row -> segment (nullable: binary search on row0)
  const int32_t *counts = nullptr;   // per-segment active rows (nullable: all)
  const void *qpart = nullptr;
  int bn = 128;                      // GEMM column tile (n-tiles per component = ceil(dp/bn))
  const void *Y = nullptr;
  double *F = nullptr;               // l (FP64): F[fidx[row]] (with fidx) or F[row]
  const int32_t *fidx = nullptr;
  void *lout = nullptr;              // l in the operand type at lout[row] when F is null
  void *grad = nullptr;              // gradient rows at goff[row] (or row * ldg)
  const int64_t *goff = nullptr;
  int64_t ldg = 0;
  void *aux = nullptr;               // responsibilities / q, row stride auxs
  int64_t auxs = 0;
};
int launch_quad_gemm_group(int dtype, const BatchDev &b, const GroupView &gv, const void *A0,
                           const void *A1, int64_t n_tiles, void *Y, void *qpart, TileCfg t,
                           hipStream_t s);
// q-partial columns per row of a problem of padded dimension dp (tile bn).
inline int group_ntn(int dp, int bn) { return (dp + bn - 1) / bn; }
int launch_finish_group(int dtype, const BatchDev &b, const FinishGroupArgs &f, hipStream_t s);
int launch_hessian_group(const BatchDev &b, const GSeg *segs, int nseg, int C, const double *Y,
                         const double *aux, int64_t auxs, const double *grad, int64_t gs,
                         const int64_t *hoff, double *H, int d_max, hipStream_t s);
int launch_beta_group(const BatchDev &b, const double *log_w, const double *logdetP,
                      double *beta, hipStream_t s);
int launch_check_group(const BatchDev &b, int ncomp, const int32_t *comp_prob,
                       const int32_t *comp_k, double *mx, int chunks, int32_t *bad,
                       hipStream_t s);
int chol_batched_u(int C, const int32_t *nv, const int64_t *off, int n_max, double *L,
                   int32_t *info, hipStream_t s);
int launch_logdet_u(int C, const int32_t *nv, const int64_t *off, const double *L,
                    const int32_t *info, double *logdet, hipStream_t s);
int launch_chol_solve_u(int C, const int32_t *nv, const int64_t *off, int n_max, const double *L,
                        const double *b, double *x, int64_t vs, const int32_t *info,
                        hipStream_t s);
size_t lbfgs_state_bytes(int dtype, int64_t B, int d, int m);
int lbfgs_carve(Arena &ar, LbfgsBuffers &b);
int launch_lbfgs_init(const LbfgsBuffers &b, const void *X0, hipStream_t s);
int launch_lbfgs_step(const LbfgsBuffers &b, int max_iter, double grad_tol, hipStream_t s);
// Steps of starts [s_begin, s_begin + count) only, dispatched for vectors of
// length at most d_class (batches sorted by dimension launch once per class).
int launch_lbfgs_step_range(const LbfgsBuffers &b, int64_t s_begin, int64_t count, int d_class,
                            double grad_tol, int max_iter, hipStream_t s);
int launch_compact(const LbfgsBuffers &b, hipStream_t s);
int launch_lbfgs_gather(const LbfgsBuffers &b, void *X, void *logl, bool logl_f64, void *grad,
                        int32_t *status, int32_t *iters, hipStream_t s);
int launch_two_loop(int64_t B, int d, int m, const int32_t *cnt, const void *S, const void *Y,
                    const void *G, void *P, int dtype, hipStream_t s);

// Dedup (leader clustering).
int dedup_run(int C, int d, const void *X, int x_dtype, const void *l, int l_dtype,
              const uint8_t *valid, double tau, int32_t *rep_of, int32_t *reps, int max_reps,
              int *n_reps, Arena &ar, hipStream_t s);
size_t dedup_ws_bytes(int C);

// Combine.
int launch_combine(int n, int d, const double *lo, const double *hi, const double *logl,
                   const double *logdet, const double *modes, int32_t *order, double *mode_log_z,
                   double *log_z, hipStream_t s);

// Whole path over a batch of n problems (host inputs; one stream).
int run_evidence_batch(int n, const sb_loglik *ll, const sb_box *box, const sb_config *cfg,
                       sb_result *res, hipStream_t s);

// Whole path (device inputs), and its workspace size.
struct DevProblem {
  int family, norm, d, K;
  const double *log_w, *mu, *prec, *lo, *hi;
  double nu, c;
};
// Identity of a captured L-BFGS iteration block: every value the block's
// launches take as an argument or that selects a kernel.  Zero-filled before
// the fields are set, so equal blocks compare equal bytewise.
struct BlockKey {
  void *stream, *ws;
  size_t ws_bytes;
  DevProblem P;
  sb_config cfg;
  double tol;
  int32_t max_iter, blk, dtype, gemm_dtype, two_stage, screen, grad_direct, hist_bf16;
  TileCfg tile, tile1, tile2;
};

// Execution state a caller keeps across whole-path calls (sb_exec): a pinned
// host word for the per-block active-count readback, phase-timing events,
// and instantiated graphs of the L-BFGS iteration block, looked up by
// BlockKey (a miss captures the block and updates the least recently used
// executable in place, or instantiates one).  Used by one call at a time.
struct ExecCtx {
  int device = -1;
  int32_t *pinned = nullptr;  // [16], hipHostMalloc
  hipEvent_t ev[10];
  bool ev_ok = false;
  static constexpr int kSlots = 4;
  struct Slot {
    bool used = false;
    BlockKey key;
    hipGraphExec_t exec = nullptr;
    uint64_t last = 0;
  } slot[kSlots];
  uint64_t tick = 0;
  int32_t n_capture = 0, n_instantiate = 0, n_update = 0, n_launch = 0;
};

// ex == nullptr: no graph, no events and no pinned memory (readbacks into
// host stack words); the phase times in res->seconds are then 0 and only the
// total is measured.  cc != nullptr: the ChiSao cycle (and the refinement
// pass when cc->n_ref > 0) replaces the single convergence phase (FP64).
int run_evidence(const DevProblem &P, const sb_config *cfg, sb_result *res, void *ws,
                 size_t ws_bytes, hipStream_t s, ExecCtx *ex,
                 const sb_chisao_config *cc = nullptr);
size_t evidence_ws_bytes(const sb_loglik *ll, const sb_config *cfg,
                         const sb_chisao_config *cc = nullptr);

// ChiSao cycle and two-pass sampling kernels (cycle.hip, chisao.hip)
int launch_normal_rows(uint64_t seed, uint32_t problem, uint32_t stream, int64_t n, int d,
                       const int32_t *rows, uint32_t i0, double *out, int64_t ld, hipStream_t s);
int launch_normalize_rows(int64_t n, int d, double *U, hipStream_t s);
int launch_gather_idx(int64_t n, int d, const int32_t *src, const double *X, double *out,
                      hipStream_t s);
int launch_scatter_idx(int64_t n, int d, const int32_t *dst, const double *in, double *X,
                       hipStream_t s);
int launch_cycle_flags(int64_t B, const uint8_t *active, const int32_t *status, const double *l,
                       uint8_t *conv, double *lmask, hipStream_t s);
int launch_mask_dead(int64_t B, const uint8_t *active, int32_t *status, hipStream_t s);
int launch_coord_spread(int64_t B, int d, const double *X, const uint8_t *free, double *sd,
                        hipStream_t s);
int launch_refine_t(int R, int n_pts, int n_ref, double delta, const double *lc, double *tref,
                    hipStream_t s);
int launch_refine_points(int R, int n_ref, int d, const double *P0, const double *P1,
                         const double *tref, double *Xr, hipStream_t s);
int launch_refine_best(int R, int n_pts, int n_ref, const double *lc, const double *lr,
                       const double *tref, double *best_l, double *best_t, hipStream_t s);
int launch_gather_starts_t(int d, int n_starts, const int32_t *start_ray, const double *best_t,
                           const double *P0, const double *P1, double *X0, hipStream_t s);
int launch_mgs_chunks(int n_chunks, int d, const int32_t *off, const int32_t *cnt, double *U,
                      hipStream_t s);

// Autotuner: tile choice for the quadratic-form GEMM (cached per shape class).
// Candidates are timed on the caller's own operands and scratch outputs
// (`probe`: the launch about to be made, whose outputs the real launch then
// overwrites), so device entry points allocate nothing.  Without a probe the
// shape is timed on private buffers only when `may_alloc` (host-level
// entry points), else the heuristic choice is returned uncached.
struct TuneProbe {
  ASrc a;
  QuadOut o;
};
TileCfg autotune_tiles(int dtype, const Model &m, int64_t M, hipStream_t s,
                       const TuneProbe *probe = nullptr, bool may_alloc = false,
                       int kt = 32);

}  // namespace sb

namespace sb {
// Batched discovery, dedup and combine (see rays.hip, dedup.hip).
int launch_rays_group(const BatchDev &b, double *P0, double *P1, float *P0f, float *P1f,
                      hipStream_t s);
int launch_ray_argmax_group(const BatchDev &b, int dtype, const void *l, double *best_l,
                            int32_t *best_j, hipStream_t s);
int launch_topn_group(const BatchDev &b, const double *best_l, int32_t *start_ray, hipStream_t s);
int launch_gather_starts_group(const BatchDev &b, const int32_t *start_ray, const int32_t *best_j,
                               const double *P0, const double *P1, void *X0, int dtype,
                               hipStream_t s);
int dedup_group_run(int n, int64_t Ctot, const int64_t *cfirst, const int64_t *ccount,
                    const BatchProb *probs, const void *X, int x_dtype, const int64_t *xoff,
                    const double *l, const uint8_t *valid, const double *ptau, int32_t *rep_of,
                    const int64_t *rbase, const int32_t *rcap, int32_t *reps, int32_t *state,
                    int64_t max_rounds, hipStream_t s);
int launch_combine_group(const BatchDev &b, const int32_t *state, const int64_t *rbase,
                         const int32_t *rcap, const int32_t *reps, const double *l,
                         const double *logdet, const double *X, const int64_t *xoff,
                         int32_t *order, double *mlz, double *log_z, hipStream_t s);
}  // namespace sb
