// Internal launcher interfaces between the gfx950 kernels and the host code.
#pragma once
#include "common.h"

namespace sb {

enum Dtype { DT_F64 = SB_DTYPE_F64, DT_F32 = SB_DTYPE_F32, DT_BF16 = SB_DTYPE_BF16 };

// Device-side view of a likelihood (all pointers are device pointers).
struct Model {
  int family = 0, norm = 0, d = 0, K = 0;
  const double *mu64 = nullptr;   // [K][d]
  const double *P64 = nullptr;    // [K][d][d]
  const double *beta = nullptr;   // [K]
  const float *mu32 = nullptr;    // [K][d] (FP32 / BF16 paths)
  const void *Plp = nullptr;      // [K][d][d] FP32 or BF16 copy
  double nu = 0.0, c = 0.0;       // Student-t dof, additive constant
};

// Source of the A operand (the points) of the quadratic-form GEMM.
struct ASrc {
  int kind = 0;                   // 0: rows of X; 1: ray points p + t (q - p)
  const void *X = nullptr;        // kind 0: [rows][ldx], double (F64) or float (F32/BF16)
  int64_t ldx = 0;
  const int32_t *rowmap = nullptr;// kind 0: GEMM row r reads X row rowmap[r] (nullable)
  const void *P0 = nullptr, *P1 = nullptr;  // kind 1: [R][d] endpoints, same type as X
  int n_pts = 1;
  bool zero_mu = false;           // A = X instead of X - mu_k
};

// Outputs of the GEMM: Y = (X - mu_k) P_k^T per component (optional) and
// per-tile partial quadratic forms sum_n delta_n Y_n.
struct QuadOut {
  void *Y = nullptr;              // [M][ldy] accumulation type, columns k*d + n
  int64_t ldy = 0;
  void *qpart = nullptr;          // [M][K][ntn]
  int ntn = 0;                    // set by the launcher (n-tiles per component)
};

// Tile shape used for a GEMM call; chosen by the autotuner.
struct TileCfg {
  int bm = 128, bn = 128;
};

int quad_gemm_ntn(int dtype, int d, TileCfg t);
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
};
int launch_finish(int dtype, const Model &m, const FinishArgs &f, hipStream_t s);

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
};
size_t lbfgs_state_bytes(int dtype, int64_t B, int d, int m);
int lbfgs_carve(Arena &ar, LbfgsBuffers &b);
int launch_lbfgs_init(const LbfgsBuffers &b, const void *X0, hipStream_t s);
int launch_lbfgs_step(const LbfgsBuffers &b, int max_iter, double grad_tol, hipStream_t s);
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

// Whole path (device inputs), and its workspace size.
struct DevProblem {
  int family, norm, d, K;
  const double *log_w, *mu, *prec, *lo, *hi;
  double nu, c;
};
int run_evidence(const DevProblem &P, const sb_config *cfg, sb_result *res, void *ws,
                 size_t ws_bytes, hipStream_t s);
size_t evidence_ws_bytes(const sb_loglik *ll, const sb_config *cfg);

// Autotuner: tile choice for the quadratic-form GEMM (cached per shape class).
TileCfg autotune_tiles(int dtype, const Model &m, int64_t M, hipStream_t s);

}  // namespace sb
