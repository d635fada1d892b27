// Quadratic-form GEMM of the likelihood families on the CDNA4 matrix cores,
// and its row epilogues (log-likelihood, hand-written gradient, HVP,
// Hessian assembly).
//
// For points x_r (rows of A) and each component k the GEMM forms
//   Y_k[r][n] = sum_j P_k[n][j] (x_r[j] - mu_k[j])      (= (P_k delta_k)_n)
// on MFMA tiles (FP64 16x16x4, FP32 16x16x4, BF16 16x16x32 with FP32
// accumulation) and, in the epilogue, the partial quadratic forms
//   qpart[r][k][tile] = sum_{n in tile} delta_k[r][n] Y_k[r][n],
// so that q_k = (x - mu_k)^T P_k (x - mu_k) is a fixed-order sum of tiles.
// The row epilogue then applies the family's closed forms: for the Gaussian
// mixture l = c + logsumexp_k(beta_k - q_k/2) and grad l = -sum_k r_k Y_k
// with r = softmax(beta - q/2); for the Student-t l = c + beta -
// ((nu+d)/2) log1p(q/nu) and grad l = -((nu+d)/(nu+q)) Y.
#include <algorithm>

#include "internal.h"
#include "mixture.h"

namespace sb {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

template <typename TOp>
struct Mfma;
template <>
struct Mfma<double> {
  using acc_t = double;
  using accv = d4v;
  static constexpr int KPI = 4;  // k per instruction
  static constexpr int KPL = 1;  // k values per lane
  // accumulator item v of lane l holds row lr + 4v (lr = l/16), column l%16
  __device__ static int row(int lr, int v) { return lr + 4 * v; }
  __device__ static accv mma(const double *a, const double *b, accv c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  using acc_t = float;
  using accv = f4v;
  static constexpr int KPI = 4;
  static constexpr int KPL = 1;
  // accumulator item v of lane l holds row 4 lr + v (lr = l/16), column l%16
  __device__ static int row(int lr, int v) { return 4 * lr + v; }
  __device__ static accv mma(const float *a, const float *b, accv c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  }
};
template <>
struct Mfma<bf16_t> {
  using acc_t = float;
  using accv = f4v;
  static constexpr int KPI = 32;
  static constexpr int KPL = 8;
  __device__ static int row(int lr, int v) { return 4 * lr + v; }
  __device__ static accv mma(const bf16_t *a, const bf16_t *b, accv c) {
    bf8v va = *reinterpret_cast<const bf8v *>(a);
    bf8v vb = *reinterpret_cast<const bf8v *>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, c, 0, 0, 0);
  }
};

template <typename TOp>
__device__ inline TOp to_op(float v);
template <>
__device__ inline float to_op<float>(float v) { return v; }
template <>
__device__ inline bf16_t to_op<bf16_t>(float v) { return f32_to_bf16(v); }
__device__ inline double to_op_d(double v) { return v; }

struct GemmParams {
  ASrc a;
  int64_t M;
  const int32_t *count;
  int d, K, ntn;
  const void *mu;  // [K][d] of type TIn
  const void *P;   // [K][d][d] of type TOp
  void *Y;
  int64_t ldy;
  void *qpart;
  GroupView gv;  // grouped mode only
  int yneg = 0;  // store -Y (a single Gaussian's gradient); q still uses Y
};

// Value of point `row` at coordinate j (type TIn), without the mean.
template <typename TIn>
__device__ inline TIn point_value(const ASrc &a, int64_t row, int64_t d, int j) {
  if (a.kind == 0) {
    int64_t r = a.rowmap ? (int64_t)a.rowmap[row] : row;
    return ((const TIn *)a.X)[r * a.ldx + j];
  }
  {
    // ray point p + t (q - p), t = (j + 1/2) / n_pts; no contraction into an
    // FMA so that the value is the same two-rounding expression everywhere.
#pragma clang fp contract(off)
    int64_t ray = row / a.n_pts;
    int jj = (int)(row % a.n_pts);
    TIn t = ((TIn)jj + (TIn)0.5) / (TIn)a.n_pts;
    TIn p = ((const TIn *)a.P0)[ray * d + j];
    TIn q = ((const TIn *)a.P1)[ray * d + j];
    return p + t * (q - p);
  }
}

template <typename TIn, typename TOp, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void quad_gemm_kernel(GemmParams g) {
  using MF = Mfma<TOp>;
  using TAcc = typename MF::acc_t;
  using accv = typename MF::accv;
  constexpr int PAD = (sizeof(TOp) == 8) ? 2 : (sizeof(TOp) == 4 ? 4 : 8);
  constexpr int LDA = BK + PAD;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  __shared__ __attribute__((aligned(16))) TOp As[BM * LDA];
  __shared__ __attribute__((aligned(16))) TOp Bs[BN * LDA];
  __shared__ TAcc qs[2][BM];

  const int64_t M = g.count ? (int64_t)(*g.count) : g.M;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  if (m0 >= M) return;
  const int k = blockIdx.y / g.ntn;
  const int n0 = (blockIdx.y % g.ntn) * BN;
  const int d = g.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const TIn *mu = g.a.zero_mu ? nullptr : (const TIn *)g.mu + (size_t)k * d;
  const TOp *Pk = (const TOp *)g.P + (size_t)k * d * d;

  accv acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = accv{0, 0, 0, 0};

  for (int k0 = 0; k0 < d; k0 += BK) {
    // A tile: delta = x - mu, converted to the operand type
    for (int e = tid; e < BM * BK; e += 256) {
      int i = e / BK, kk = e % BK;
      int64_t row = m0 + i;
      int j = k0 + kk;
      TIn v = 0;
      if (row < M && j < d) {
        v = point_value<TIn>(g.a, row, d, j);
        if (mu) v = v - mu[j];
      }
      if constexpr (sizeof(TOp) == 8)
        As[i * LDA + kk] = v;
      else
        As[i * LDA + kk] = to_op<TOp>((float)v);
    }
    // B tile: rows n of P_k (Bs[n][j] = P_k[n0+n][k0+j]) so Y_n = sum_j P[n][j] delta_j
    for (int e = tid; e < BN * BK; e += 256) {
      int n = e / BK, kk = e % BK;
      int nn = n0 + n, j = k0 + kk;
      TOp v;
      if (nn < d && j < d)
        v = Pk[(size_t)nn * d + j];
      else
        v = TOp(0);
      Bs[n * LDA + kk] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += MF::KPI) {
      const int kl = kk + MF::KPL * (lane >> 4);
      const TOp *af[TM];
      const TOp *bfp[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = &As[(wm * WM + i * 16 + (lane & 15)) * LDA + kl];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfp[j] = &Bs[(wn * WN + j * 16 + (lane & 15)) * LDA + kl];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(af[i], bfp[j], acc[i][j]);
    }
    __syncthreads();
  }

  // Epilogue: store Y, accumulate delta * Y per row over this tile's columns.
  const int lr = lane >> 4, lc = lane & 15;
  TAcc qrow[TM][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) qrow[i][v] = 0;
  TAcc *Y = (TAcc *)g.Y;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int il = wm * WM + i * 16 + MF::row(lr, v);
      const int64_t row = m0 + il;
      if (row >= M) continue;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = n0 + wn * WN + j * 16 + lc;
        if (n >= d) continue;
        TAcc yv = acc[i][j][v];
        if (Y) Y[row * g.ldy + (int64_t)k * d + n] = g.yneg ? -yv : yv;
        TIn x = point_value<TIn>(g.a, row, d, n);
        TAcc dl = (TAcc)(mu ? x - mu[n] : x);
        qrow[i][v] += dl * yv;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      TAcc t = qrow[i][v];
      t += __shfl_xor(t, 1, 64);
      t += __shfl_xor(t, 2, 64);
      t += __shfl_xor(t, 4, 64);
      t += __shfl_xor(t, 8, 64);
      qrow[i][v] = t;
    }
  if (lc == 0) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) qs[wn][wm * WM + i * 16 + MF::row(lr, v)] = qrow[i][v];
  }
  __syncthreads();
  if (g.qpart) {
    TAcc *qp = (TAcc *)g.qpart;
    for (int i = tid; i < BM; i += 256) {
      int64_t row = m0 + i;
      if (row < M) qp[(row * g.K + k) * g.ntn + (blockIdx.y % g.ntn)] = qs[0][i] + qs[1][i];
    }
  }
}

int quad_gemm_ntn(int dtype, int d, TileCfg t) { return (int)ceil_div(d, t.bn); }

template <typename TIn, typename TOp, int BM, int BN, int BK>
static int launch_scalar(const GemmParams &p, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(p.M, BM), (unsigned)(p.K * p.ntn));
  if (grid.x == 0 || grid.y == 0) return SB_OK;
  hipLaunchKernelGGL((quad_gemm_kernel<TIn, TOp, BM, BN, BK>), grid, dim3(256), 0, s, p);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// ------------------------------------------------------- vectorised GEMM
//
// Same tile, fragment and epilogue layout as quad_gemm_kernel, for d a
// multiple of the 16-byte vector widths: every thread owns fixed A rows and
// B rows for the whole K loop (row pointers and the row map resolved once),
// loads 16-byte vectors, and prefetches k-tile t+1 into registers while the
// MFMAs of tile t run from LDS.

template <typename T>
struct V16;
template <>
struct V16<double> {
  typedef double v __attribute__((ext_vector_type(2)));
  static constexpr int N = 2;
};
template <>
struct V16<float> {
  typedef float v __attribute__((ext_vector_type(4)));
  static constexpr int N = 4;
};
template <>
struct V16<bf16_t> {
  typedef uint16_t v __attribute__((ext_vector_type(8)));
  static constexpr int N = 8;
};

template <typename TIn, typename TOp, int BM, int BN, int BK, int KIND, bool GROUP>
__global__ __launch_bounds__(256) void quad_gemm_vec_kernel(GemmParams g) {
  using MF = Mfma<TOp>;
  using TAcc = typename MF::acc_t;
  using accv = typename MF::accv;
  using VI = typename V16<TIn>::v;
  using VO = typename V16<TOp>::v;
  constexpr int NI = V16<TIn>::N, NO = V16<TOp>::N;
  constexpr int PAD = (sizeof(TOp) == 8) ? 2 : (sizeof(TOp) == 4 ? 4 : 8);
  constexpr int LDA = BK + PAD;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int VRA = BK / NI, VRB = BK / NO;
  constexpr int NA = BM * VRA / 256, NB = BN * VRB / 256;
  static_assert(NA >= 1 && NB >= 1 && (BM * VRA) % 256 == 0 && (BN * VRB) % 256 == 0, "tile");
  static_assert(256 % VRA == 0 && 256 % VRB == 0, "tile");
  __shared__ __attribute__((aligned(16))) TOp As[BM * LDA];
  __shared__ __attribute__((aligned(16))) TOp Bs[BN * LDA];
  __shared__ TAcc qs[2][BM];

  // ---- tile context: rows [m0, M) (global row indices), component k, columns n0..
  int64_t M, m0;
  int k, nt, ntn, d, n_pts;
  const TIn *mu;
  const TOp *Pk;
  const TIn *X0 = (const TIn *)g.a.X;      // kind 0 rows / kind 1 ray start points
  const TIn *X1 = (const TIn *)g.a.P1;     // kind 1 ray end points
  int64_t pt_first = 0, roff = 0;          // kind 1: first point row, endpoint base
  int64_t ybase = 0, qbase = 0;            // grouped: packed Y / q-partial bases
  int64_t ystr = 0, qstr = 0;              // grouped: Y / q-partial row strides
  if constexpr (!GROUP) {
    M = g.count ? (int64_t)(*g.count) : g.M;
    m0 = (int64_t)blockIdx.x * BM;
    if (m0 >= M) return;
    ntn = g.ntn;
    k = blockIdx.y / ntn;
    nt = blockIdx.y % ntn;
    d = g.d;
    n_pts = g.a.n_pts;
    mu = g.a.zero_mu ? nullptr : (const TIn *)g.mu + (size_t)k * d;
    Pk = (const TOp *)g.P + (size_t)k * d * d;
    if constexpr (KIND == 1) X0 = (const TIn *)g.a.P0;
  } else {
    const GroupView &gv = g.gv;
    const int sgi = gv.tile_seg[blockIdx.x];
    const GSeg sg = gv.segs[sgi];
    const BatchProb pr = gv.probs[sg.prob];
    const int64_t rows = gv.counts ? (int64_t)gv.counts[sgi] : (int64_t)sg.rows;
    m0 = sg.row0 + (int64_t)gv.tile_idx[blockIdx.x] * BM;
    M = sg.row0 + rows;
    if (m0 >= M) return;
    d = pr.dp;
    ntn = (d + BN - 1) / BN;
    if ((int)blockIdx.y >= pr.K * ntn) return;
    k = blockIdx.y / ntn;
    nt = blockIdx.y % ntn;
    n_pts = pr.n_pts;
    mu = g.a.zero_mu ? nullptr : (const TIn *)gv.mu + pr.mu_off + (size_t)k * d;
    Pk = (const TOp *)gv.P + pr.P_off + (size_t)k * d * d;
    // packed Y / q-partial rows of this segment
    ystr = (int64_t)pr.K * d;
    qstr = (int64_t)pr.K * ntn;
    ybase = sg.yoff - sg.row0 * ystr;
    qbase = sg.qoff - sg.row0 * qstr;
    if constexpr (KIND == 1) {
      X0 = (const TIn *)g.a.P0;
      pt_first = sg.row0;
      roff = pr.roff0;
    }
  }
  const int n0 = nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Row pointers of global row `row`: its X row (kind 0) or its ray's two
  // endpoints and parameter t (kind 1).
  auto row_src = [&](int64_t row, const TIn *&a, const TIn *&b, TIn &t) {
    if constexpr (KIND == 0) {
      int64_t off;
      if constexpr (GROUP)
        off = g.gv.rowoff[row];
      else
        off = (g.a.rowmap ? (int64_t)g.a.rowmap[row] : row) * g.a.ldx;
      a = X0 + off;
      b = nullptr;
      t = 0;
    } else {
      const int64_t i = row - pt_first;
      const int64_t ray = i / n_pts;
      const int jj = (int)(i % n_pts);
      t = ((TIn)jj + (TIn)0.5) / (TIn)n_pts;
      a = X0 + roff + ray * d;
      b = X1 + roff + ray * d;
    }
  };

  // fixed rows of this thread
  const int ca = tid % VRA, cb = tid % VRB;
  const TIn *arow[NA];
  const TIn *qrow_p[NA];
  TIn tpar[NA];
  bool aok[NA];
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    const int i = (tid + 256 * r) / VRA;
    const int64_t row = m0 + i;
    aok[r] = row < M;
    arow[r] = nullptr;
    qrow_p[r] = nullptr;
    tpar[r] = 0;
    if (aok[r]) row_src(row, arow[r], qrow_p[r], tpar[r]);
  }
  const TOp *brow[NB];
  bool bok[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    const int n = (tid + 256 * r) / VRB;
    bok[r] = (n0 + n) < d;
    brow[r] = Pk + (size_t)(n0 + n) * d;
  }

  VI ra[NA], rq[NA], rmu;
  VO rb[NB];
  auto zero_i = []() {
    VI z;
#pragma unroll
    for (int e = 0; e < NI; ++e) z[e] = (TIn)0;
    return z;
  };
  auto zero_o = []() {
    VO z;
#pragma unroll
    for (int e = 0; e < NO; ++e) z[e] = 0;
    return z;
  };
  auto load = [&](int k0) {
    const int ka = k0 + ca * NI;
    const bool kin = ka < d;
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      const bool ok = aok[r] && kin;
      ra[r] = ok ? *(const VI *)(arow[r] + ka) : zero_i();
      if constexpr (KIND == 1) rq[r] = ok ? *(const VI *)(qrow_p[r] + ka) : zero_i();
    }
    rmu = (mu && kin) ? *(const VI *)(mu + ka) : zero_i();
    const int kb = k0 + cb * NO;
    const bool kbin = kb < d;
#pragma unroll
    for (int r = 0; r < NB; ++r) rb[r] = (bok[r] && kbin) ? *(const VO *)(brow[r] + kb) : zero_o();
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      const int i = (tid + 256 * r) / VRA;
      TOp *dst = &As[i * LDA + ca * NI];
#pragma unroll
      for (int e = 0; e < NI; ++e) {
        TIn x;
        if constexpr (KIND == 0) {
          x = ra[r][e];
        } else {
#pragma clang fp contract(off)
          x = ra[r][e] + tpar[r] * (rq[r][e] - ra[r][e]);
        }
        const TIn v = aok[r] ? x - rmu[e] : (TIn)0;
        if constexpr (sizeof(TOp) == 8)
          dst[e] = v;
        else
          dst[e] = to_op<TOp>((float)v);
      }
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int n = (tid + 256 * r) / VRB;
      *(VO *)&Bs[n * LDA + cb * NO] = rb[r];
    }
  };

  accv acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = accv{0, 0, 0, 0};

  load(0);
  for (int k0 = 0; k0 < d; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < d) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += MF::KPI) {
      const int kl = kk + MF::KPL * (lane >> 4);
      const TOp *af[TM];
      const TOp *bfp[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = &As[(wm * WM + i * 16 + (lane & 15)) * LDA + kl];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfp[j] = &Bs[(wn * WN + j * 16 + (lane & 15)) * LDA + kl];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(af[i], bfp[j], acc[i][j]);
    }
    __syncthreads();
  }

  // Epilogue: store Y, partial q per row for this tile's columns.
  const int lr = lane >> 4, lc = lane & 15;
  TAcc qrow[TM][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) qrow[i][v] = 0;
  TAcc *Y = (TAcc *)g.Y;
  const int64_t ystride = GROUP ? ystr : g.ldy;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int il = wm * WM + i * 16 + MF::row(lr, v);
      const int64_t row = m0 + il;
      if (row >= M) continue;
      const TIn *pa, *pb;
      TIn tt;
      row_src(row, pa, pb, tt);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = n0 + wn * WN + j * 16 + lc;
        if (n >= d) continue;
        TAcc yv = acc[i][j][v];
        if (Y) Y[ybase + row * ystride + (int64_t)k * d + n] = g.yneg ? -yv : yv;
        TIn x;
        if constexpr (KIND == 0) {
          x = pa[n];
        } else {
#pragma clang fp contract(off)
          x = pa[n] + tt * (pb[n] - pa[n]);
        }
        TAcc dl = (TAcc)(mu ? x - mu[n] : x);
        qrow[i][v] += dl * yv;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      TAcc t = qrow[i][v];
      t += __shfl_xor(t, 1, 64);
      t += __shfl_xor(t, 2, 64);
      t += __shfl_xor(t, 4, 64);
      t += __shfl_xor(t, 8, 64);
      qrow[i][v] = t;
    }
  if (lc == 0) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) qs[wn][wm * WM + i * 16 + MF::row(lr, v)] = qrow[i][v];
  }
  __syncthreads();
  if (g.qpart) {
    TAcc *qp = (TAcc *)g.qpart;
    for (int i = tid; i < BM; i += 256) {
      const int64_t row = m0 + i;
      if (row >= M) continue;
      if constexpr (GROUP)
        qp[qbase + row * qstr + (int64_t)k * ntn + nt] = qs[0][i] + qs[1][i];
      else
        qp[(row * g.K + k) * g.ntn + nt] = qs[0][i] + qs[1][i];
    }
  }
}

template <typename TIn, typename TOp, int BM, int BN, int BK>
static int launch_t(const GemmParams &p, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(p.M, BM), (unsigned)(p.K * p.ntn));
  if (grid.x == 0 || grid.y == 0) return SB_OK;
  // vector path: 16-byte aligned rows of X (or ray endpoints), mu and P
  const bool vec = (p.d % V16<TIn>::N == 0) && (p.d % V16<TOp>::N == 0) &&
                   (p.a.kind == 1 || p.a.ldx % V16<TIn>::N == 0);
  if (vec && p.a.kind == 0)
    hipLaunchKernelGGL((quad_gemm_vec_kernel<TIn, TOp, BM, BN, BK, 0, false>), grid, dim3(256), 0, s, p);
  else if (vec)
    hipLaunchKernelGGL((quad_gemm_vec_kernel<TIn, TOp, BM, BN, BK, 1, false>), grid, dim3(256), 0, s, p);
  else
    return launch_scalar<TIn, TOp, BM, BN, BK>(p, s);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int launch_quad_gemm(int dtype, const Model &m, const ASrc &a, int64_t M, const int32_t *count,
                     QuadOut &o, TileCfg t, hipStream_t s) {
  if (a.kind == 1 && a.dt > 0.f &&
      !((dtype == DT_F32S || dtype == DT_BF16) && quad_gemm_bf16_ok(m.d))) {
    set_error("ray nodes need the BF16 matrix-core kernel (d = %d)", m.d);
    return SB_E_UNSUPPORTED;
  }
  // BF16 matrix-core kernel: split FP32 always when d allows (else plain
  // FP32), BF16 when d allows and the BF16 copy is given.
  if (dtype == DT_F32S && quad_gemm_bf16_ok(m.d))
    return launch_quad_gemm_bf16(3, m, a, M, count, o, s, t);
  if (dtype == DT_F32S) dtype = DT_F32;
  if (dtype == DT_BF16 && quad_gemm_bf16_ok(m.d)) {
    Model mb = m;
    if (!mb.Phi) mb.Phi = (const bf16_t *)m.Plp;
    return launch_quad_gemm_bf16(1, mb, a, M, count, o, s, t);
  }
  if (o.ymap || o.sumsq || o.gcnt) {
    set_error("row-mapped, grouped or sum-of-squares outputs need the BF16 matrix-core kernel");
    return SB_E_UNSUPPORTED;
  }
  GemmParams p;
  p.a = a;
  p.M = M;
  p.count = count;
  p.d = m.d;
  p.K = m.K;
  p.yneg = o.yneg ? 1 : 0;
  if (t.bn != 64 && t.bn != 128) t.bn = 128;
  // (32-row tiles: FP64 with a 32-wide k-tile and 64 columns only)
  const bool f64_32 = dtype == DT_F64 && t.bm == 32 && t.bn == 64 && t.bk == 32;
  if (t.bm != 64 && t.bm != 128 && !f64_32) t.bm = 128;
  o.ntn = (int)ceil_div(m.d, t.bn);
  p.ntn = o.ntn;
  p.Y = o.Y;
  p.ldy = o.ldy;
  p.qpart = o.qpart;
  if (dtype == DT_F64) {
    p.mu = m.mu64;
    p.P = m.P64;
    if (t.bk == 32) {  // 32-wide k-tiles: half the barriers per MFMA
      if (f64_32) return launch_t<double, double, 32, 64, 32>(p, s);
      if (t.bm == 64 && t.bn == 64) return launch_t<double, double, 64, 64, 32>(p, s);
      if (t.bm == 128 && t.bn == 64) return launch_t<double, double, 128, 64, 32>(p, s);
      if (t.bm == 64 && t.bn == 128) return launch_t<double, double, 64, 128, 32>(p, s);
    }
    if (t.bm == 64 && t.bn == 64) return launch_t<double, double, 64, 64, 16>(p, s);
    if (t.bm == 128 && t.bn == 64) return launch_t<double, double, 128, 64, 16>(p, s);
    if (t.bm == 64 && t.bn == 128) return launch_t<double, double, 64, 128, 16>(p, s);
    return launch_t<double, double, 128, 128, 16>(p, s);
  }
  p.mu = m.mu32;
  p.P = m.Plp;
  if (!p.P || !p.mu) {
    set_error("low-precision model copies missing");
    return SB_E_INVAL;
  }
  if (dtype == DT_F32) {
    if (t.bk == 32) {  // 32-wide k-tiles: half the barriers per MFMA
      if (t.bm == 64 && t.bn == 64) return launch_t<float, float, 64, 64, 32>(p, s);
      if (t.bm == 128 && t.bn == 64) return launch_t<float, float, 128, 64, 32>(p, s);
      if (t.bm == 64 && t.bn == 128) return launch_t<float, float, 64, 128, 32>(p, s);
      return launch_t<float, float, 128, 128, 32>(p, s);
    }
    if (t.bm == 64 && t.bn == 64) return launch_t<float, float, 64, 64, 16>(p, s);
    if (t.bm == 128 && t.bn == 64) return launch_t<float, float, 128, 64, 16>(p, s);
    if (t.bm == 64 && t.bn == 128) return launch_t<float, float, 64, 128, 16>(p, s);
    return launch_t<float, float, 128, 128, 16>(p, s);
  }
  if (t.bm == 64 && t.bn == 64) return launch_t<float, bf16_t, 64, 64, 32>(p, s);
  if (t.bm == 128 && t.bn == 64) return launch_t<float, bf16_t, 128, 64, 32>(p, s);
  if (t.bm == 64 && t.bn == 128) return launch_t<float, bf16_t, 64, 128, 32>(p, s);
  return launch_t<float, bf16_t, 128, 128, 32>(p, s);
}

// ------------------------------------------------------------------ finish

// One wave per row: q_k from the tile partials, the family's l, and (if
// requested) the gradient -sum_k r_k Y_k (mixture) or -((nu+d)/(nu+q)) Y.
// The scalar part (q_k sums, beta_k - q_k/2, logsumexp, responsibilities)
// runs in FP64 for every operand type: l carries constants of size
// ~(d/2) log 2 pi and (1/2) log det P, and the line search compares l values
// whose difference is far below the FP32 spacing at that magnitude.
template <typename T>
__global__ __launch_bounds__(256) void finish_kernel(Model m, FinishArgs f) {
  const int64_t M = f.count ? (int64_t)(*f.count) : f.M;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= M) return;
  const int d = m.d, K = m.K;
  const T *qp = (const T *)f.qpart + (size_t)row * K * f.ntn;
  const T *Y = (const T *)f.Y + (size_t)row * f.ldy;
  const int64_t orow = f.outmap ? (int64_t)f.outmap[row] : row;
  T *gout = f.grad ? (T *)f.grad + (size_t)orow * f.ldg : nullptr;
  if (m.family == SB_FAMILY_STUDENT_T) {
    double q = 0;
    for (int t = 0; t < f.ntn; ++t) q += (double)qp[t];
    const double nd = m.nu + (double)d;
    const double l = m.c + m.beta[0] - 0.5 * nd * log1p(q / m.nu);
    if (lane == 0) {
      if (f.logl_f64)
        ((double *)f.logl)[orow] = l;
      else
        ((T *)f.logl)[orow] = (T)l;
      if (f.aux) ((T *)f.aux)[row * K] = (T)q;
    }
    if (gout) {
      const T sc = (T)(nd / (m.nu + q));
      constexpr int V = 16 / sizeof(T);
      typedef T vt __attribute__((ext_vector_type(V)));
      if (d % V == 0 && ((uintptr_t)Y % 16) == 0 && ((uintptr_t)gout % 16) == 0) {
        for (int n = lane * V; n < d; n += 64 * V) {
          vt y = *(const vt *)&Y[n];
#pragma unroll
          for (int e = 0; e < V; ++e) y[e] = -sc * y[e];
          *(vt *)&gout[n] = y;
        }
      } else {
        for (int n = lane; n < d; n += 64) gout[n] = -sc * Y[n];
      }
    }
    return;
  }
  // (its gradient written by the contraction: one listed component, r = 1)
  if (f.resp && f.skip1 && __popc(f.skip1[row]) == 1) return;
  T r[kMaxK];
  if (f.resp) {  // l and the responsibilities came from the mixture-rows pass
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) r[k] = (k < K) ? (T)((const float *)f.resp)[row * K + k] : (T)0;
  } else {
    double lse;
    mixture_resp<T>(m, qp, f.ntn, lse, r);
    if (lane == 0) {
      if (f.logl_f64)
        ((double *)f.logl)[orow] = m.c + lse;
      else
        ((T *)f.logl)[orow] = (T)(m.c + lse);
    }
  }
  if (f.aux && lane < K) {
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k == lane) ((T *)f.aux)[row * K + k] = r[k];
  }
  if (gout) {
    // components whose responsibility rounds to zero in T add nothing: their
    // Y rows are not read (separated mixtures touch one row of K).  16-byte
    // accesses where the rows allow them (same sums, element by element).
    constexpr int V = 16 / sizeof(T);
    typedef T vt __attribute__((ext_vector_type(V)));
    const bool vec = d % V == 0 && ((uintptr_t)Y % 16) == 0 && ((uintptr_t)gout % 16) == 0;
    if (vec) {
      for (int n = lane * V; n < d; n += 64 * V) {
        vt s;
#pragma unroll
        for (int e = 0; e < V; ++e) s[e] = 0;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
          if (k < K && r[k] != (T)0) {
            const vt y = *(const vt *)&Y[(size_t)k * d + n];
#pragma unroll
            for (int e = 0; e < V; ++e) s[e] += r[k] * y[e];
          }
#pragma unroll
        for (int e = 0; e < V; ++e) s[e] = -s[e];
        *(vt *)&gout[n] = s;
      }
    } else {
      for (int n = lane; n < d; n += 64) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
          if (k < K && r[k] != (T)0) s += r[k] * Y[(size_t)k * d + n];
        gout[n] = -s;
      }
    }
  }
}

// Mixture rows (FP32 operands), one thread per row: l = c + logsumexp_k
// (beta_k - q_k/2) and the responsibilities r_k (the epilogue's own function,
// FP64 arithmetic, r stored in FP32); per component k the rows with r_k != 0
// are appended to rows[k] (GEMM row) and xrows[k] (operand row: rowmap[r] or
// r), cnt[k] (zeroed by the caller) counting them.  The epilogue then takes
// r from `resp`, so it reads exactly the Y rows formed for these lists.
// Order within a list is arbitrary; every row's outputs are independent of it.
__global__ __launch_bounds__(256) void mixture_rows_kernel(Model m, MixRowsArgs a) {
  const int64_t Mr = a.count ? (int64_t)(*a.count) : a.M;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= Mr) return;
  const int K = m.K;
  double lse;
  float r[kMaxK];
  mixture_resp<float>(m, a.qpart + (size_t)row * K * a.ntn, a.ntn, lse, r);
  const int64_t orow = a.outmap ? (int64_t)a.outmap[row] : row;
  if (a.logl_f64)
    ((double *)a.logl)[orow] = m.c + lse;
  else
    ((float *)a.logl)[orow] = (float)(m.c + lse);
#pragma unroll
  for (int k = 0; k < kMaxK; ++k)
    if (k < K) {
      a.resp[row * K + k] = r[k];
      if (r[k] != 0.f) {
        const int pos = atomicAdd(&a.cnt[k], 1);
        a.rows[(int64_t)k * a.cap + pos] = (int32_t)row;
        a.xrows[(int64_t)k * a.cap + pos] = a.rowmap ? a.rowmap[row] : (int32_t)row;
      }
    }
}

int launch_mixture_rows(const Model &m, const MixRowsArgs &a, hipStream_t s) {
  if (m.K > kMaxK || m.family != SB_FAMILY_GAUSS_MIX) {
    set_error("mixture rows: Gaussian mixtures of at most %d components", kMaxK);
    return SB_E_UNSUPPORTED;
  }
  if (a.M > a.cap || a.M > 0x7fffffffll) {
    set_error("mixture rows: %lld rows over the capacity %lld", (long long)a.M, (long long)a.cap);
    return SB_E_INVAL;
  }
  if (a.M <= 0) return SB_OK;
  // (one wave per workgroup: the rows spread over every CU)
  hipLaunchKernelGGL(mixture_rows_kernel, dim3((unsigned)ceil_div(a.M, 64)), dim3(64), 0, s, m, a);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Screened mixture rows.  With U_k^T U_k = P_k, s_k(x) = sqrt(q_k(x)) =
// |U_k (x - mu_k)| is Lipschitz with constant |U_k|_2 <= sigma_k =
// sqrt(rho_k), rho_k the largest absolute row sum of P_k (Gershgorin).  A row
// keeps bounds lb_k <= s_k(x_ref) <= ub_k at its last evaluated point, so at x
//   max(0, lb_k - sigma_k D) <= s_k(x) <= ub_k + sigma_k D,  D = |x - x_ref|,
// which brackets a_k = beta_k - q_k / 2 in [lo_k, hi_k].  Component k is
// dropped when hi_k < max_j lo_j - kScreenGap: its exact responsibility is
// then below e^-kScreenGap, far under FP32's smallest subnormal (e^-103.3),
// and its share of l far below FP64 resolution; it keeps the widened bounds.
// A listed component gets new bounds from the split contraction's q_k, whose
// error is at most c_q rho_k |x - mu_k|^2: the split representation drops
// 3 2^-16 of each |P_nj delta_j|, FP32 accumulation of the 3d products and
// of the d-term q sum at most (d + 32) 2^-24 each, and |delta|^T |P| |delta|
// <= rho |delta|^2 (c_q has a 1.25 margin); s_k of the rounded delta =
// fl32(x - mu_k) is within sigma_k 2^-23 |delta| of s_k(x).  A NaN anywhere
// keeps the component (the comparisons fail).
constexpr double kScreenGap = 120.0;

__device__ inline double screen_cq(int d) {
  return 1.25 * (3.0 * 0x1p-16 + 4.0 * (d + 32) * 0x1p-24);
}
// relative slack of FP32 sums of d squares
__device__ inline double screen_rq(int d) { return (2.0 * d + 128) * 0x1p-24; }
__device__ inline double clamp0(double v) {  // max(v, 0), NaN stays NaN
  return v > 0.0 ? v : (v <= 0.0 ? 0.0 : (double)NAN);
}

// One wave per row: |x - x_ref|^2 over the row, the decision (the row's
// component mask), the dropped components' widened bounds and q partials,
// |x - mu_k|^2 of the listed ones, and x_ref = x.  NX > 0 (d <= 256 NX): the
// row's x and x_ref sit in registers, NX 16-byte chunks per lane, their loads
// and the bounds' issued together, and x is read once; NX = 0: any d, the row
// streamed twice.  Both forms sum in the same order.
template <int NX>
__global__ __launch_bounds__(256) void mixture_screen_kernel(Model m, ScreenArgs a) {
  // the list pass (the next launch) counts into cnt: zero it here
  if (blockIdx.x == 0 && threadIdx.x < m.K) a.cnt[threadIdx.x] = 0;
  const int64_t Mr = a.count ? (int64_t)(*a.count) : a.M;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= Mr) return;
  const int d = m.d, K = m.K;
  const int32_t xr = a.rowmap ? a.rowmap[row] : (int32_t)row;
  const float *x = a.X + (int64_t)xr * a.ldx;
  float *xref = a.xref + (int64_t)xr * d;
  const bool href = a.hasref[xr] > 0;
  constexpr int NR = NX > 0 ? NX : 1;
  f4v xv[NR], rv[NR];
  if constexpr (NX > 0) {
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int j = 4 * lane + 256 * i;  // (d % 8 == 0: a chunk is whole or absent)
      xv[i] = rv[i] = f4v{0.f, 0.f, 0.f, 0.f};
      if (j < d) {
        xv[i] = *(const f4v *)(x + j);
        if (href) rv[i] = __builtin_nontemporal_load((const f4v *)(xref + j));
      }
    }
  }
  uint32_t keep = (1u << K) - 1u;  // (K <= 16) no reference yet: every component
  if (href) {
    // component k's bounds in lane k
    double *lb = a.bnd + (int64_t)xr * 2 * K, *ub = lb + K;
    const bool act = lane < K;
    const double L0 = act ? lb[lane] : 0.0, U0 = act ? ub[lane] : 0.0;
    float dd = 0.f;
    if constexpr (NX > 0) {
#pragma unroll
      for (int i = 0; i < NX; ++i)
        if (4 * lane + 256 * i < d)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float t = xv[i][e] - rv[i][e];
            dd += t * t;
          }
    } else {
      for (int j = 4 * lane; j < d; j += 256) {  // (d % 8 == 0, 16-byte rows)
        const f4v xw = *(const f4v *)(x + j);
        const f4v rw = __builtin_nontemporal_load((const f4v *)(xref + j));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float t = xw[e] - rw[e];
          dd += t * t;
        }
      }
    }
    // (the butterfly leaves the same sum in every lane: the decision is uniform)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dd += __shfl_xor(dd, o, 64);
    const double D = sqrt((double)dd * (1.0 + screen_rq(d))) * (1.0 + 0x1p-40);
    double Lk = 0.0, Uk = 0.0, hi = -INFINITY;
    if (act) {
      const double w = sqrt(a.rho[lane] * (1.0 + 0x1p-40)) * D;
      Lk = clamp0(L0 - w);
      Uk = U0 + w;
      hi = m.beta[lane] - 0.5 * Uk * Uk;
    }
    // largest upper end over the components (fmax drops a NaN: the maximum of
    // the others, as a running fmax over k would give)
    double mx = hi;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    const bool kb = act && !(m.beta[lane] - 0.5 * Lk * Lk < mx - kScreenGap);
    keep = (uint32_t)__ballot(kb);
    // dropped: the widened bounds now hold at x
    if (act && !kb) {
      lb[lane] = Lk;
      ub[lane] = Uk;
    }
  }
  // |x - mu_k|^2 of the listed components (for their new bounds) and x_ref = x
  float nrm[kMaxK];
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) nrm[k] = 0.f;
  auto chunk = [&](int j, const f4v &xw) {
    __builtin_nontemporal_store(xw, (f4v *)(xref + j));
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < K && ((keep >> k) & 1u)) {
        const f4v mv = *(const f4v *)(m.mu32 + (int64_t)k * d + j);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float t = xw[e] - mv[e];  // delta as the contraction forms it
          nrm[k] += t * t;
        }
      }
  };
  if constexpr (NX > 0) {
#pragma unroll
    for (int i = 0; i < NX; ++i)
      if (4 * lane + 256 * i < d) chunk(4 * lane + 256 * i, xv[i]);
  } else {
    for (int j = 4 * lane; j < d; j += 256) chunk(j, *(const f4v *)(x + j));
  }
#pragma unroll
  for (int k = 0; k < kMaxK; ++k)
    if (k < K && ((keep >> k) & 1u))
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) nrm[k] += __shfl_xor(nrm[k], o, 64);
#pragma unroll
  for (int k = 0; k < kMaxK; ++k)
    if (k == lane && k < K) a.nrm[row * K + k] = nrm[k];
  if (lane == 0) a.mask[row] = keep;
  // a dropped component's q partials: +inf, 0, ... (one coalesced row block)
  float *q2 = a.qpart + (size_t)row * K * a.ntn;
  for (int i = lane; i < K * a.ntn; i += 64)
    if (!((keep >> (i / a.ntn)) & 1u)) q2[i] = (i % a.ntn == 0) ? INFINITY : 0.f;
}

// Lists from the masks, one thread per row, 1024 rows per workgroup: ranks
// within each wave by ballot, wave offsets in LDS, one atomic per workgroup
// and component (same-address atomics from many workgroups serialise).
__global__ __launch_bounds__(1024) void mixture_lists_kernel(Model m, ScreenArgs a) {
  __shared__ int woff[16][kMaxK];
  __shared__ int base[kMaxK];
  const int64_t Mr = a.count ? (int64_t)(*a.count) : a.M;
  const int64_t row = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int K = m.K;
  const bool valid = row < Mr;
  const uint32_t mk = valid ? a.mask[row] : 0u;
  int rank[kMaxK];
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) {
    rank[k] = 0;
    if (k < K) {
      const uint64_t bal = __ballot((mk >> k) & 1u);
      rank[k] = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) woff[wave][k] = __popcll(bal);
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    const int k = threadIdx.x;
    int tot = 0;
    for (int w = 0; w < 16; ++w) {
      const int c = woff[w][k];
      woff[w][k] = tot;
      tot += c;
    }
    base[k] = tot ? atomicAdd(&a.cnt[k], tot) : 0;
  }
  __syncthreads();
  if (!valid) return;
  const int32_t xr = a.rowmap ? a.rowmap[row] : (int32_t)row;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k)
    if (k < K && ((mk >> k) & 1u)) {
      const int64_t pos = (int64_t)k * a.cap + base[k] + woff[wave][k] + rank[k];
      a.rows[pos] = (int32_t)row;
      a.xrows[pos] = xr;
      if (a.gdst)
        a.gdst[pos] = __popc(mk) == 1 ? (a.outmap ? a.outmap[row] : (int32_t)row) : -1;
    }
}

// After the contraction, 16 lanes per row with component k in lane k of the
// row's group: l and the responsibilities from q, the arithmetic of the
// epilogue's own function (mixture_resp) in its order: lane k sums q_k's
// tile partials in turn and forms exp(a_k - max), and every lane adds the
// gathered terms over k = 0, 1, ...; r stored in FP32.  Then the listed
// components' bounds from their q_k.
__global__ __launch_bounds__(256) void mixture_post_kernel(Model m, ScreenArgs a) {
  static_assert(kMaxK <= 16, "a row's components fit its 16 lanes");
  const int64_t Mr = a.count ? (int64_t)(*a.count) : a.M;
  const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int c = threadIdx.x & 15, base = (threadIdx.x & 63) & ~15;
  if (row >= Mr) return;  // (whole groups: the shuffles below stay in the group)
  const int d = m.d, K = m.K;
  const bool act = c < K;
  const float *qp = a.qpart + (size_t)row * K * a.ntn;
  double q = 0.0, ak = 0.0;
  if (act) {
    for (int t = 0; t < a.ntn; ++t) q += (double)qp[c * a.ntn + t];
    ak = m.beta[c] - 0.5 * q;
  }
  double lse;
  if (K == 1) {
    lse = __shfl(ak, base, 64);
  } else {
    double mx = -INFINITY;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
      const double v = __shfl(ak, base + k, 64);
      if (k < K) mx = fmax(mx, v);
    }
    const double ek = act ? exp(ak - mx) : 0.0;
    double ssum = 0;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
      const double v = __shfl(ek, base + k, 64);
      if (k < K) ssum += v;
    }
    lse = mx + log(ssum);
  }
  if (c == 0) {
    const int64_t orow = a.outmap ? (int64_t)a.outmap[row] : row;
    if (a.logl_f64)
      ((double *)a.logl)[orow] = m.c + lse;
    else
      ((float *)a.logl)[orow] = (float)(m.c + lse);
  }
  if (act) a.resp[row * K + c] = K == 1 ? 1.f : (float)exp(ak - lse);
  const int32_t xr = a.rowmap ? a.rowmap[row] : (int32_t)row;
  const uint32_t mk = a.mask[row];
  if (act && ((mk >> c) & 1u)) {
    const double cq = screen_cq(d), rq = screen_rq(d);
    double *lb = a.bnd + (int64_t)xr * 2 * K, *ub = lb + K;
    const double rk = a.rho[c] * (1.0 + 0x1p-40);
    const double nk = (double)a.nrm[row * K + c] * (1.0 + rq);
    const double e = cq * rk * nk;
    // (+- sigma_k 2^-23 |delta|: delta = fl32(x - mu_k) against the exact x - mu_k)
    const double rr = sqrt(rk * nk) * 0x1p-23;
    lb[c] = clamp0(sqrt(clamp0(q - e)) - rr);
    ub[c] = sqrt(clamp0(q + e)) + rr;
  }
  if (c == 0) a.hasref[xr] = 1;
}

static int screen_check(const Model &m, const ScreenArgs &a, const char *what) {
  if (m.K > kMaxK || m.K > 64 || m.family != SB_FAMILY_GAUSS_MIX) {
    set_error("%s: Gaussian mixtures of at most %d components", what, kMaxK);
    return SB_E_UNSUPPORTED;
  }
  if (a.M > a.cap || a.M > 0x7fffffffll) {
    set_error("%s: %lld rows over the capacity %lld", what, (long long)a.M, (long long)a.cap);
    return SB_E_INVAL;
  }
  if (m.d % 8 != 0 || (uintptr_t)a.X % 16 != 0 || a.ldx % 4 != 0 ||
      (uintptr_t)m.mu32 % 16 != 0 || (uintptr_t)a.xref % 16 != 0 || !a.rho || !a.bnd ||
      !a.hasref || !a.nrm || !a.qpart || a.ntn < 1 || !a.mask) {
    set_error("%s: needs d %% 8 == 0, 16-byte rows and the screening state", what);
    return SB_E_INVAL;
  }
  if (a.nstate < a.M) {
    set_error("%s: %lld operand rows with state for %lld rows", what, (long long)a.nstate,
              (long long)a.M);
    return SB_E_INVAL;
  }
  return SB_OK;
}

int launch_mixture_screen(const Model &m, const ScreenArgs &a, hipStream_t s) {
  int st = screen_check(m, a, "mixture screen");
  if (st) return st;
  if (!a.cnt || !a.rows || !a.xrows) {
    set_error("mixture screen: needs the component lists");
    return SB_E_INVAL;
  }
  if (a.M <= 0) return launch_fill_i32(m.K, 0, a.cnt, s);  // empty lists
  const dim3 grid((unsigned)ceil_div(a.M, 4));
  switch (ceil_div(m.d, 256)) {
    case 1: hipLaunchKernelGGL(mixture_screen_kernel<1>, grid, dim3(256), 0, s, m, a); break;
    case 2: hipLaunchKernelGGL(mixture_screen_kernel<2>, grid, dim3(256), 0, s, m, a); break;
    case 3: hipLaunchKernelGGL(mixture_screen_kernel<3>, grid, dim3(256), 0, s, m, a); break;
    case 4: hipLaunchKernelGGL(mixture_screen_kernel<4>, grid, dim3(256), 0, s, m, a); break;
    default: hipLaunchKernelGGL(mixture_screen_kernel<0>, grid, dim3(256), 0, s, m, a); break;
  }
  SB_LAUNCH_CHECK();
  hipLaunchKernelGGL(mixture_lists_kernel, dim3((unsigned)ceil_div(a.M, 1024)), dim3(1024), 0, s,
                     m, a);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int launch_mixture_post(const Model &m, const ScreenArgs &a, hipStream_t s) {
  int st = screen_check(m, a, "mixture post");
  if (st || a.M <= 0) return st;
  if (!a.logl || !a.resp) {
    set_error("mixture post: needs l and responsibility outputs");
    return SB_E_INVAL;
  }
  hipLaunchKernelGGL(mixture_post_kernel, dim3((unsigned)ceil_div(a.M, 16)), dim3(256), 0, s, m,
                     a);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// One wave per row of P_k: the absolute row sum, folded into rho[k] with an
// integer max on the bit pattern (order-preserving for non-negative doubles).
__global__ __launch_bounds__(256) void row_abs_max_kernel(int K, int d, const double *P,
                                                          double *rho) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= (int64_t)K * d) return;
  const double *p = P + r * d;
  double t = 0.0;
  for (int j = lane; j < d; j += 64) t += fabs(p[j]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o, 64);
  if (lane == 0)
    atomicMax((unsigned long long *)&rho[r / d], (unsigned long long)__double_as_longlong(t));
}

// Power steps, batched over the K matrices: w = P v (one wave per row), then
// theta = v . w, v = w / |w| (one workgroup per matrix).
__global__ __launch_bounds__(256) void pw_gemv_kernel(int K, int d, const double *P,
                                                      const double *v, double *w) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= (int64_t)K * d) return;
  const int64_t k = r / d;
  const double *p = P + r * d, *vk = v + k * d;
  double t = 0.0;
  for (int j = lane; j < d; j += 64) t += p[j] * vk[j];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o, 64);
  if (lane == 0) w[r] = t;
}

__global__ __launch_bounds__(256) void pw_norm_kernel(int d, double *v, const double *w,
                                                      double *theta, int init) {
  const int k = blockIdx.x;
  double *vk = v + (int64_t)k * d;
  const double *wk = w + (int64_t)k * d;
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double x = init ? 1.0 : wk[i];
    a += x * x;
    b += init ? 0.0 : vk[i] * wk[i];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0][0]);
  if (threadIdx.x == 0) theta[k] = red[1][0];
  for (int i = threadIdx.x; i < d; i += 256) vk[i] = (init ? 1.0 : wk[i]) * inv;
}

// A_k = 1.25 theta_k I - P_k
__global__ void pw_shift_kernel(int K, int d, const double *P, const double *theta, double *A) {
  const int64_t n = (int64_t)K * d * d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = i / ((int64_t)d * d), rc = i % ((int64_t)d * d);
    const int r = (int)(rc / d), c = (int)(rc % d);
    A[i] = (r == c ? 1.25 * theta[k] : 0.0) - P[i];
  }
}

__global__ void pw_pick_kernel(int K, const double *theta, const int32_t *info, double *rho) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double tau = 1.25 * theta[k] * (1.0 + 0x1p-20);
  if (info[k] == 0 && tau > 0.0 && tau < rho[k]) rho[k] = tau;
}

int launch_lmax_bound(int K, int d, const double *P, double *rho, double *work, double *A,
                      int32_t *info, hipStream_t s) {
  if (K <= 0 || d <= 0) return SB_OK;
  double *v = work, *w = work + (int64_t)K * d, *theta = work + 2 * (int64_t)K * d;
  hipLaunchKernelGGL(pw_norm_kernel, dim3((unsigned)K), dim3(256), 0, s, d, v, w, theta, 1);
  SB_LAUNCH_CHECK();
  for (int it = 0; it < 16; ++it) {
    hipLaunchKernelGGL(pw_gemv_kernel, dim3((unsigned)ceil_div((int64_t)K * d, 4)), dim3(256), 0,
                       s, K, d, P, v, w);
    SB_LAUNCH_CHECK();
    hipLaunchKernelGGL(pw_norm_kernel, dim3((unsigned)K), dim3(256), 0, s, d, v, w, theta, 0);
    SB_LAUNCH_CHECK();
  }
  const int64_t n = (int64_t)K * d * d;
  hipLaunchKernelGGL(pw_shift_kernel, dim3((unsigned)std::min<int64_t>(8192, ceil_div(n, 256))),
                     dim3(256), 0, s, K, d, P, theta, A);
  SB_LAUNCH_CHECK();
  int st = chol_batched(K, d, A, A, info, s);
  if (st) return st;
  hipLaunchKernelGGL(pw_pick_kernel, dim3((unsigned)ceil_div(K, 64)), dim3(64), 0, s, K, theta,
                     info, rho);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int launch_row_abs_max(int K, int d, const double *P, double *rho, hipStream_t s) {
  if (K <= 0 || d <= 0) return SB_OK;
  int st = launch_fill_i32(2 * (int64_t)K, 0, (int32_t *)rho, s);
  if (st) return st;
  hipLaunchKernelGGL(row_abs_max_kernel, dim3((unsigned)ceil_div((int64_t)K * d, 4)), dim3(256),
                     0, s, K, d, P, rho);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Ray-point scores from three nodes per ray.  Along a ray the quadratic
// form q_k(t) = (p + t (q - p) - mu_k)^T P_k (p + t (q - p) - mu_k) is a
// polynomial of degree two in t, so its values at t = 0, 1/2, 1 fix it and
// Lagrange interpolation gives q_k at every sample t_j = (j + 1/2) / n_pts
// (weights at most 1.25 in absolute sum on [0, 1]: the node errors are not
// amplified).  RB rays per workgroup: node sums into LDS, then one thread
// per sample point for the family's l, in FP64 as in the row epilogue.
constexpr int kNodeRays = 8;
__global__ __launch_bounds__(256) void ray_nodes_finish_kernel(Model m, int64_t R, int n_pts,
                                                               int ntn, const float *qpart,
                                                               float *l) {
  __shared__ double qn[kNodeRays][3][kMaxK];
  const int K = m.K;
  const int64_t r0 = (int64_t)blockIdx.x * kNodeRays;
  for (int i = threadIdx.x; i < kNodeRays * 3 * K; i += blockDim.x) {
    const int rb = i / (3 * K), node = (i / K) % 3, k = i % K;
    const int64_t r = r0 + rb;
    double q = 0.0;
    if (r < R) {
      const float *qp = qpart + ((size_t)(3 * r + node) * K + k) * ntn;
      for (int t = 0; t < ntn; ++t) q += (double)qp[t];
    }
    qn[rb][node][k] = q;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kNodeRays * n_pts; i += blockDim.x) {
    const int rb = i / n_pts, j = i % n_pts;
    const int64_t r = r0 + rb;
    if (r >= R) break;  // (later i only reach later rays)
    const double t = ((double)j + 0.5) / (double)n_pts;
    // Lagrange weights of the nodes 0, 1/2, 1
    const double w0 = 2.0 * (t - 0.5) * (t - 1.0), w1 = -4.0 * t * (t - 1.0),
                 w2 = 2.0 * t * (t - 0.5);
    double out;
    if (m.family == SB_FAMILY_STUDENT_T) {
      const double q = w0 * qn[rb][0][0] + w1 * qn[rb][1][0] + w2 * qn[rb][2][0];
      out = m.c + m.beta[0] - 0.5 * (m.nu + (double)m.d) * log1p(q / m.nu);
    } else {
      double a[kMaxK];
      double mx = -INFINITY;
#pragma unroll
      for (int k = 0; k < kMaxK; ++k) {
        if (k < K) {
          const double q = w0 * qn[rb][0][k] + w1 * qn[rb][1][k] + w2 * qn[rb][2][k];
          a[k] = m.beta[k] - 0.5 * q;
          mx = fmax(mx, a[k]);
        }
      }
      double lse = a[0];
      if (K > 1) {
        double ssum = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
          if (k < K) ssum += exp(a[k] - mx);
        lse = mx + log(ssum);
      }
      out = m.c + lse;
    }
    l[r * n_pts + j] = (float)out;
  }
}

int launch_ray_nodes_finish(const Model &m, int64_t R, int n_pts, int ntn, const float *qpart,
                            float *l, hipStream_t s) {
  if (R <= 0) return SB_OK;
  if (n_pts < 1 || ntn < 1 || m.K < 1 || m.K > kMaxK || !qpart || !l) {
    set_error("ray nodes: bad arguments");
    return SB_E_INVAL;
  }
  hipLaunchKernelGGL(ray_nodes_finish_kernel, dim3((unsigned)ceil_div(R, kNodeRays)), dim3(256),
                     0, s, m, R, n_pts, ntn, qpart, l);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int discover_bf16_nodes(const Model &m, const float *P0, const float *P1, int R, int n_pts,
                        float *qpart, float *l, hipStream_t s) {
  if (!quad_gemm_bf16_ok(m.d)) {
    set_error("ray nodes need the BF16 matrix-core kernel (d = %d)", m.d);
    return SB_E_UNSUPPORTED;
  }
  ASrc a;
  a.kind = 1;
  a.P0 = P0;
  a.P1 = P1;
  a.n_pts = 3;
  a.t0 = 0.f;
  a.dt = 0.5f;
  QuadOut o;
  o.Y = nullptr;
  o.ldy = (int64_t)m.K * m.d;
  o.qpart = qpart;
  const int64_t M = 3ll * R;
  const TuneProbe pr{a, o};
  TileCfg t = autotune_tiles(DT_BF16, m, M, s, &pr);
  int st = launch_quad_gemm(DT_BF16, m, a, M, nullptr, o, t, s);
  if (st) return st;
  return launch_ray_nodes_finish(m, R, n_pts, o.ntn, qpart, l, s);
}

int launch_finish(int dtype, const Model &m, const FinishArgs &f, hipStream_t s) {
  if (m.K > kMaxK) {
    set_error("K=%d exceeds the supported %d components", m.K, kMaxK);
    return SB_E_UNSUPPORTED;
  }
  if (f.skip1 && (!f.resp || f.aux)) {
    set_error("finish: skipped rows need precomputed responsibilities and no aux output");
    return SB_E_INVAL;
  }
  dim3 grid((unsigned)ceil_div(f.M, 4));
  if (grid.x == 0) return SB_OK;
  if (dtype == DT_F64)
    hipLaunchKernelGGL(finish_kernel<double>, grid, dim3(256), 0, s, m, f);
  else
    hipLaunchKernelGGL(finish_kernel<float>, grid, dim3(256), 0, s, m, f);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// -------------------------------------------------------------------- HVP

// HV = nabla^2 l v.  Mixture: sum_k r_k (Y_k (Y_k . v) - Z_k) - g (g . v)
// with Y_k = P_k delta_k, Z_k = P_k v, g = grad l.  Student-t:
// -((nu+d)/(nu+q)) Z + (2 (nu+d)/(nu+q)^2) Y (Y . v).  One wave per row.
__global__ __launch_bounds__(256) void hvp_finish_kernel(Model m, HvpArgs h) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= h.M) return;
  const int d = m.d, K = m.K;
  const double *qp = (const double *)h.qpart + (size_t)row * K * h.ntn;
  const double *Y = h.Y + (size_t)row * h.ldy;
  const double *Z = h.Z + (size_t)row * h.ldy;
  const double *v = h.V + (size_t)row * d;
  double *out = h.HV + (size_t)row * d;
  if (m.family == SB_FAMILY_STUDENT_T) {
    double q = 0;
    for (int t = 0; t < h.ntn; ++t) q += qp[t];
    double nd = m.nu + d, den = m.nu + q;
    double uv = 0;
    for (int n = lane; n < d; n += 64) uv += Y[n] * v[n];
    uv = wave_sum(uv);
    for (int n = lane; n < d; n += 64)
      out[n] = -(nd / den) * Z[n] + (2.0 * nd / (den * den)) * Y[n] * uv;
    return;
  }
  double a[kMaxK], r[kMaxK], uv[kMaxK];
  double mx = -INFINITY;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) {
    if (k < K) {
      double q = 0;
      for (int t = 0; t < h.ntn; ++t) q += qp[k * h.ntn + t];
      a[k] = m.beta[k] - 0.5 * q;
      mx = fmax(mx, a[k]);
    }
  }
  double ssum = 0;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k)
    if (k < K) ssum += exp(a[k] - mx);
  double lse = mx + log(ssum);
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) r[k] = (k < K) ? (K == 1 ? 1.0 : exp(a[k] - lse)) : 0.0;
  // g . v and Y_k . v
  double gv = 0;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) uv[k] = 0;
  for (int n = lane; n < d; n += 64) {
    double gn = 0;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < K) {
        gn += r[k] * Y[(size_t)k * d + n];
        uv[k] += Y[(size_t)k * d + n] * v[n];
      }
    gv += -gn * v[n];
  }
  gv = wave_sum(gv);
#pragma unroll
  for (int k = 0; k < kMaxK; ++k)
    if (k < K) uv[k] = wave_sum(uv[k]);
  for (int n = lane; n < d; n += 64) {
    double gn = 0;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < K) gn += r[k] * Y[(size_t)k * d + n];
    gn = -gn;
    double hv = -gn * gv;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < K) hv += r[k] * (Y[(size_t)k * d + n] * uv[k] - Z[(size_t)k * d + n]);
    out[n] = hv;
  }
}

int launch_hvp_finish(const Model &m, const HvpArgs &h, hipStream_t s) {
  if (m.K > kMaxK) return SB_E_UNSUPPORTED;
  dim3 grid((unsigned)ceil_div(h.M, 4));
  if (grid.x == 0) return SB_OK;
  hipLaunchKernelGGL(hvp_finish_kernel, grid, dim3(256), 0, s, m, h);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// --------------------------------------------------------- Hessian assembly

// H = -nabla^2 l = sum_k r_k (P_k - u_k u_k^T) + g g^T (mixture) or
// ((nu+d)/(nu+q)) P - (2 (nu+d)/(nu+q)^2) u u^T (Student-t), u_k = Y_k;
// symmetrised as (H + H^T)/2.  This is the HVP epilogue with V = I.
__device__ inline double hess_entry(const Model &m, int c, int i, int j, const double *Y,
                                    int64_t ldy, const double *aux, const double *grad) {
  const int d = m.d, K = m.K;
  const double *y = Y + (size_t)c * ldy;
  if (m.family == SB_FAMILY_STUDENT_T) {
    double q = aux[(size_t)c * K];
    double nd = m.nu + d, den = m.nu + q;
    return (nd / den) * m.P64[(size_t)i * d + j] - (2.0 * nd / (den * den)) * y[i] * y[j];
  }
  const double *g = grad + (size_t)c * d;
  double s = g[i] * g[j];
  for (int k = 0; k < K; ++k) {
    double rk = aux[(size_t)c * K + k];
    const double *u = y + (size_t)k * d;
    s += rk * (m.P64[(size_t)k * d * d + (size_t)i * d + j] - u[i] * u[j]);
  }
  return s;
}

__global__ __launch_bounds__(256) void hessian_kernel(Model m, int C, const double *Y, int64_t ldy,
                                                      const double *aux, const double *grad,
                                                      double *H) {
  const int c = blockIdx.z;
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int d = m.d;
  if (c >= C || i >= d || j >= d) return;
  double hij = hess_entry(m, c, i, j, Y, ldy, aux, grad);
  double hji = hess_entry(m, c, j, i, Y, ldy, aux, grad);
  H[(size_t)c * d * d + (size_t)i * d + j] = 0.5 * (hij + hji);
}

int launch_hessian_assemble(const Model &m, int C, const double *Y, int64_t ldy,
                            const double *aux, const double *grad, double *H, hipStream_t s) {
  if (C <= 0) return SB_OK;
  dim3 grid((unsigned)ceil_div(m.d, 16), (unsigned)ceil_div(m.d, 16), (unsigned)C);
  hipLaunchKernelGGL(hessian_kernel, grid, dim3(256), 0, s, m, C, Y, ldy, aux, grad, H);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// ---------------------------------------------------------------- prep

__global__ void convert_model_kernel(const double *P, const double *mu, int64_t nP, int64_t nmu,
                                     float *P32, bf16_t *Pbf, float *mu32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = i; e < nP; e += stride) {
    float v = (float)P[e];
    if (P32) P32[e] = v;
    if (Pbf) Pbf[e] = f32_to_bf16(v);
  }
  for (int64_t e = i; e < nmu; e += stride)
    if (mu32) mu32[e] = (float)mu[e];
}

int launch_convert_model(const Model &m, float *P32, bf16_t *Pbf, float *mu32, hipStream_t s) {
  int64_t nP = (int64_t)m.K * m.d * m.d, nmu = (int64_t)m.K * m.d;
  unsigned blocks = (unsigned)std::min<int64_t>(4096, ceil_div(nP, 256));
  hipLaunchKernelGGL(convert_model_kernel, dim3(blocks), dim3(256), 0, s, m.P64, m.mu64, nP, nmu,
                     P32, Pbf, mu32);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Per-component max |P_k| into mx[k], then bad[0] = 1 if any
// |P_ij - P_ji| > 1e-12 * mx[k].
// max |P_k| over (chunks x K) workgroups: each reduces a strided share and
// folds it in with an integer atomic max on the bit pattern (non-negative
// doubles order like their bits; a NaN entry yields a NaN-pattern maximum).
__global__ void zero_f64_kernel(int n, double *x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}
__global__ __launch_bounds__(256) void maxabs_kernel(const double *P, int d, double *mx) {
  const int k = blockIdx.y;
  const double *Pk = P + (size_t)k * d * d;
  __shared__ double red[4];
  double v = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)d * d;
       e += (int64_t)gridDim.x * 256)
    v = fmax(v, fabs(Pk[e]));
  v = block_max<256>(v, red);
  if (threadIdx.x == 0)
    atomicMax((unsigned long long *)&mx[k], (unsigned long long)__double_as_longlong(v));
}
__global__ void symmetry_kernel(const double *P, int d, const double *mx, int32_t *bad) {
  const int k = blockIdx.y;
  const double *Pk = P + (size_t)k * d * d;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  int i = (int)(e / d), j = (int)(e % d);
  if (j <= i) return;
  double a = Pk[(size_t)i * d + j], b = Pk[(size_t)j * d + i];
  if (!(fabs(a - b) <= 1e-12 * mx[k])) bad[0] = 1;
}

int launch_symmetry_check(const double *P, int K, int d, double *mx, int32_t *bad,
                          hipStream_t s) {
  hipLaunchKernelGGL(zero_f64_kernel, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, s, K, mx);
  const unsigned chunks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, ceil_div((int64_t)d * d, 4096)));
  hipLaunchKernelGGL(maxabs_kernel, dim3(chunks, K), dim3(256), 0, s, P, d, mx);
  SB_LAUNCH_CHECK();
  dim3 grid((unsigned)ceil_div((int64_t)d * d, 256), (unsigned)K);
  hipLaunchKernelGGL(symmetry_kernel, grid, dim3(256), 0, s, P, d, mx, bad);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// beta_k from log w_k and log det P_k (see sb.h for the closed forms).
__global__ void beta_kernel(Model m, const double *log_w, const double *logdetP, double *beta) {
  const int k = threadIdx.x;
  if (k >= m.K) return;
  const double d = m.d;
  double b = 0.0;
  if (m.family == SB_FAMILY_GAUSS_MIX) {
    b = log_w ? log_w[k] : 0.0;
    if (m.norm == SB_NORM_DENSITY) b += 0.5 * logdetP[k] - 0.5 * d * kLog2Pi;
  } else if (m.norm == SB_NORM_DENSITY) {
    b = lgamma(0.5 * (m.nu + d)) - lgamma(0.5 * m.nu) - 0.5 * d * log(m.nu * M_PI) +
        0.5 * logdetP[k];
  }
  beta[k] = b;
}

int launch_beta(const Model &m, const double *log_w, const double *logdetP, double *beta,
                hipStream_t s) {
  hipLaunchKernelGGL(beta_kernel, dim3(1), dim3(64 * (int)ceil_div(m.K, 64)), 0, s, m, log_w,
                     logdetP, beta);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// ---------------------------------------------------------------- casts

__global__ void cast_d2f(int64_t n, const double *a, float *b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = (float)a[i];
}
__global__ void cast_f2d(int64_t n, const float *a, double *b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = (double)a[i];
}
__global__ void fill_i32(int64_t n, int32_t v, int32_t *p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
int launch_cast_f64_f32(int64_t n, const double *a, float *b, hipStream_t s) {
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(cast_d2f, dim3((unsigned)std::min<int64_t>(8192, ceil_div(n, 256))),
                     dim3(256), 0, s, n, a, b);
  SB_LAUNCH_CHECK();
  return SB_OK;
}
int launch_cast_f32_f64(int64_t n, const float *a, double *b, hipStream_t s) {
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(cast_f2d, dim3((unsigned)std::min<int64_t>(8192, ceil_div(n, 256))),
                     dim3(256), 0, s, n, a, b);
  SB_LAUNCH_CHECK();
  return SB_OK;
}
int launch_fill_i32(int64_t n, int32_t v, int32_t *p, hipStream_t s) {
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(fill_i32, dim3((unsigned)std::min<int64_t>(8192, ceil_div(n, 256))),
                     dim3(256), 0, s, n, v, p);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb

// ====================================================================
// Batched (grouped) variants: many problems of uneven dimension, each
// M-tile belonging to one problem; see BatchProb.
namespace sb {

int launch_quad_gemm_group(int dtype, const BatchDev &b, const GroupView &gv_in, const void *A0,
                           const void *A1, int64_t n_tiles, void *Y, void *qpart, TileCfg t,
                           hipStream_t s) {
  if (n_tiles <= 0) return SB_OK;
  GemmParams p{};
  p.a.kind = gv_in.kind;
  p.a.X = A0;
  p.a.P0 = A0;
  p.a.P1 = A1;
  p.Y = Y;
  p.qpart = qpart;
  p.gv = gv_in;
  const int bn = (t.bn == 64) ? 64 : 128;
  const int bm = (t.bm == 64) ? 64 : 128;
  dim3 grid((unsigned)n_tiles, (unsigned)(b.K_max * ceil_div(b.dp_max, bn)));
  if (dtype == DT_F64) {
    p.gv.mu = b.mu64;
    p.gv.P = b.P64;
  } else if (dtype == DT_F32) {
    p.gv.mu = b.mu32;
    p.gv.P = b.P32;
  } else {
    p.gv.mu = b.mu32;
    p.gv.P = b.Pbf;
  }
#define SB_GG(TI, TO, BMv, BNv, BKv)                                                             \
  do {                                                                                           \
    if (p.a.kind == 0)                                                                           \
      hipLaunchKernelGGL((quad_gemm_vec_kernel<TI, TO, BMv, BNv, BKv, 0, true>), grid, dim3(256), \
                         0, s, p);                                                               \
    else                                                                                         \
      hipLaunchKernelGGL((quad_gemm_vec_kernel<TI, TO, BMv, BNv, BKv, 1, true>), grid, dim3(256), \
                         0, s, p);                                                               \
  } while (0)
  if (dtype == DT_F64) {
    if (bm == 64 && bn == 64) SB_GG(double, double, 64, 64, 16);
    else if (bm == 128 && bn == 64) SB_GG(double, double, 128, 64, 16);
    else if (bm == 64) SB_GG(double, double, 64, 128, 16);
    else SB_GG(double, double, 128, 128, 16);
  } else if (dtype == DT_F32) {
    if (bm == 64 && bn == 64) SB_GG(float, float, 64, 64, 16);
    else if (bm == 128 && bn == 64) SB_GG(float, float, 128, 64, 16);
    else if (bm == 64) SB_GG(float, float, 64, 128, 16);
    else SB_GG(float, float, 128, 128, 16);
  } else {
    if (bm == 64 && bn == 64) SB_GG(float, bf16_t, 64, 64, 32);
    else if (bm == 128 && bn == 64) SB_GG(float, bf16_t, 128, 64, 32);
    else if (bm == 64) SB_GG(float, bf16_t, 64, 128, 32);
    else SB_GG(float, bf16_t, 128, 128, 32);
  }
#undef SB_GG
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Segment of global row r: the last segment whose row0 <= r.
__device__ inline int find_seg(const GSeg *segs, int n, int64_t r) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].row0 <= r)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Row epilogue for a batch (one wave per row), same arithmetic as
// finish_kernel.  l -> F[fidx[r]] / F[r] (FP64) or lout[r] (type T);
// gradient -> grad + goff[r] (or r * ldg); aux -> aux + r * auxs.
template <typename T>
__global__ __launch_bounds__(256) void finish_group_kernel(BatchDev b, FinishGroupArgs f) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= f.nrows) return;
  const int sgi = f.rowseg ? f.rowseg[row] : find_seg(f.segs, f.nseg, row);
  const GSeg sg = f.segs[sgi];
  const int64_t rows = f.counts ? (int64_t)f.counts[sgi] : (int64_t)sg.rows;
  if (row - sg.row0 >= rows) return;
  const BatchProb pr = b.probs[sg.prob];
  const int d = pr.dp, K = pr.K;
  const int ntn = (d + f.bn - 1) / f.bn;
  const int64_t rl = row - sg.row0;
  const T *qp = (const T *)f.qpart + sg.qoff + rl * (int64_t)K * ntn;
  const T *Y = f.Y ? (const T *)f.Y + sg.yoff + rl * (int64_t)K * d : nullptr;
  const double *beta = b.beta + pr.beta_off;
  T *gout = nullptr;
  if (f.grad) gout = (T *)f.grad + (f.goff ? f.goff[row] : row * (int64_t)f.ldg);
  auto put_l = [&](double l) {
    if (lane != 0) return;
    if (f.F)
      f.F[f.fidx ? (int64_t)f.fidx[row] : row] = l;
    else
      ((T *)f.lout)[row] = (T)l;
  };
  if (pr.family == SB_FAMILY_STUDENT_T) {
    double q = 0;
    for (int t = 0; t < ntn; ++t) q += (double)qp[t];
    const double nd = pr.nu + (double)pr.d;
    put_l(pr.c + beta[0] - 0.5 * nd * log1p(q / pr.nu));
    if (f.aux && lane == 0) ((T *)f.aux)[row * f.auxs] = (T)q;
    if (gout) {
      const T sc = (T)(nd / (pr.nu + q));
      for (int n = lane; n < d; n += 64) gout[n] = -sc * Y[n];
    }
    return;
  }
  double a[kMaxK];
  double mx = -INFINITY;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) {
    if (k < K) {
      double q = 0;
      for (int t = 0; t < ntn; ++t) q += (double)qp[k * ntn + t];
      a[k] = beta[k] - 0.5 * q;
      mx = fmax(mx, a[k]);
    }
  }
  double lse;
  if (K == 1) {
    lse = a[0];
  } else {
    double ssum = 0;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < K) ssum += exp(a[k] - mx);
    lse = mx + log(ssum);
  }
  put_l(pr.c + lse);
  T r[kMaxK];
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) r[k] = (k < K) ? (K == 1 ? (T)1 : (T)exp(a[k] - lse)) : (T)0;
  if (f.aux && lane < K) {
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k == lane) ((T *)f.aux)[row * f.auxs + k] = r[k];
  }
  if (gout) {
    // components whose responsibility rounds to zero in T add nothing: their
    // Y rows are not read (separated mixtures touch one row of K).  16-byte
    // accesses where the rows allow them (same sums, element by element).
    constexpr int V = 16 / sizeof(T);
    typedef T vt __attribute__((ext_vector_type(V)));
    const bool vec = d % V == 0 && ((uintptr_t)Y % 16) == 0 && ((uintptr_t)gout % 16) == 0;
    if (vec) {
      for (int n = lane * V; n < d; n += 64 * V) {
        vt s;
#pragma unroll
        for (int e = 0; e < V; ++e) s[e] = 0;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
          if (k < K && r[k] != (T)0) {
            const vt y = *(const vt *)&Y[(size_t)k * d + n];
#pragma unroll
            for (int e = 0; e < V; ++e) s[e] += r[k] * y[e];
          }
#pragma unroll
        for (int e = 0; e < V; ++e) s[e] = -s[e];
        *(vt *)&gout[n] = s;
      }
    } else {
      for (int n = lane; n < d; n += 64) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
          if (k < K && r[k] != (T)0) s += r[k] * Y[(size_t)k * d + n];
        gout[n] = -s;
      }
    }
  }
}

int launch_finish_group(int dtype, const BatchDev &b, const FinishGroupArgs &f, hipStream_t s) {
  if (b.K_max > kMaxK) {
    set_error("K=%d exceeds the supported %d components", b.K_max, kMaxK);
    return SB_E_UNSUPPORTED;
  }
  if (f.nrows <= 0 || f.nseg <= 0) return SB_OK;
  dim3 grid((unsigned)ceil_div(f.nrows, 4));
  if (dtype == DT_F64)
    hipLaunchKernelGGL(finish_group_kernel<double>, grid, dim3(256), 0, s, b, f);
  else
    hipLaunchKernelGGL(finish_group_kernel<float>, grid, dim3(256), 0, s, b, f);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Hessian H = -nabla^2 l of row c (its segment's problem), true dimension
// d_p, leading dimension d_p, at H + hoff[c]; Y rows packed by segment,
// aux rows of stride auxs, gradient rows of stride gs.  Symmetrised.
__global__ __launch_bounds__(256) void hessian_group_kernel(BatchDev b, const GSeg *segs,
                                                             int nseg, int C, const double *Y,
                                                             const double *aux, int64_t auxs,
                                                             const double *grad, int64_t gs,
                                                             const int64_t *hoff, double *H) {
  const int c = blockIdx.z;
  if (c >= C) return;
  const GSeg sg = segs[find_seg(segs, nseg, c)];
  const BatchProb pr = b.probs[sg.prob];
  const int d = pr.d, dp = pr.dp;
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  if (i >= d || j >= d) return;
  const double *y = Y + sg.yoff + (int64_t)(c - sg.row0) * pr.K * dp;
  const double *P = b.P64 + pr.P_off;
  auto entry = [&](int a, int bb) -> double {
    if (pr.family == SB_FAMILY_STUDENT_T) {
      const double q = aux[(size_t)c * auxs];
      const double nd = pr.nu + pr.d, den = pr.nu + q;
      return (nd / den) * P[(size_t)a * dp + bb] - (2.0 * nd / (den * den)) * y[a] * y[bb];
    }
    const double *g = grad + (size_t)c * gs;
    double s = g[a] * g[bb];
    for (int k = 0; k < pr.K; ++k) {
      const double rk = aux[(size_t)c * auxs + k];
      const double *u = y + (size_t)k * dp;
      s += rk * (P[(size_t)k * dp * dp + (size_t)a * dp + bb] - u[a] * u[bb]);
    }
    return s;
  };
  H[hoff[c] + (size_t)i * d + j] = 0.5 * (entry(i, j) + entry(j, i));
}

int launch_hessian_group(const BatchDev &b, const GSeg *segs, int nseg, int C, const double *Y,
                         const double *aux, int64_t auxs, const double *grad, int64_t gs,
                         const int64_t *hoff, double *H, int d_max, hipStream_t s) {
  if (C <= 0) return SB_OK;
  dim3 grid((unsigned)ceil_div(d_max, 16), (unsigned)ceil_div(d_max, 16), (unsigned)C);
  hipLaunchKernelGGL(hessian_group_kernel, grid, dim3(256), 0, s, b, segs, nseg, C, Y, aux, auxs,
                     grad, gs, hoff, H);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// beta_k of every problem (one thread per component).
__global__ void beta_group_kernel(BatchDev b, const double *log_w, const double *logdetP,
                                  double *beta) {
  const int p = blockIdx.x;
  const BatchProb pr = b.probs[p];
  const int k = threadIdx.x;
  if (k >= pr.K) return;
  const double d = pr.d;
  const int64_t o = pr.beta_off + k;
  double v = 0.0;
  if (pr.family == SB_FAMILY_GAUSS_MIX) {
    v = log_w ? log_w[o] : 0.0;
    if (pr.norm == SB_NORM_DENSITY) v += 0.5 * logdetP[o] - 0.5 * d * kLog2Pi;
  } else if (pr.norm == SB_NORM_DENSITY) {
    v = lgamma(0.5 * (pr.nu + d)) - lgamma(0.5 * pr.nu) - 0.5 * d * log(pr.nu * M_PI) +
        0.5 * logdetP[o];
  }
  beta[o] = v;
}

int launch_beta_group(const BatchDev &b, const double *log_w, const double *logdetP,
                      double *beta, hipStream_t s) {
  hipLaunchKernelGGL(beta_group_kernel, dim3(b.n), dim3(64 * (int)ceil_div(b.K_max, 64)), 0, s,
                     b, log_w, logdetP, beta);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Per component: max |P| (for the FP32 tolerance) and the symmetry flag, in
// the padded layout (padding is zero and symmetric).  grid (chunks, components).
__global__ __launch_bounds__(256) void maxabs_sym_group_kernel(BatchDev b, const int32_t *comp_prob,
                                                               const int32_t *comp_k, double *mx,
                                                               int32_t *bad) {
  const int c = blockIdx.y;
  const BatchProb pr = b.probs[comp_prob[c]];
  const int dp = pr.dp;
  const double *P = b.P64 + pr.P_off + (size_t)comp_k[c] * dp * dp;
  __shared__ double red[4];
  const int64_t n = (int64_t)dp * dp;
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    m = fmax(m, fabs(P[e]));
  m = block_max<256>(m, red);
  if (threadIdx.x == 0) mx[(size_t)c * gridDim.x + blockIdx.x] = m;
}
__global__ __launch_bounds__(256) void sym_group_kernel(BatchDev b, const int32_t *comp_prob,
                                                        const int32_t *comp_k, const double *mx,
                                                        int chunks, int32_t *bad) {
  const int c = blockIdx.y;
  const BatchProb pr = b.probs[comp_prob[c]];
  const int dp = pr.dp;
  const double *P = b.P64 + pr.P_off + (size_t)comp_k[c] * dp * dp;
  double m = 0.0;
  for (int t = 0; t < chunks; ++t) m = fmax(m, mx[(size_t)c * chunks + t]);
  const int64_t n = (int64_t)dp * dp;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / dp), j = (int)(e % dp);
    if (j <= i) continue;
    if (!(fabs(P[e] - P[(size_t)j * dp + i]) <= 1e-12 * m)) bad[0] = 1;
  }
}

int launch_check_group(const BatchDev &b, int ncomp, const int32_t *comp_prob,
                       const int32_t *comp_k, double *mx, int chunks, int32_t *bad,
                       hipStream_t s) {
  if (ncomp <= 0) return SB_OK;
  hipLaunchKernelGGL(maxabs_sym_group_kernel, dim3(chunks, ncomp), dim3(256), 0, s, b, comp_prob,
                     comp_k, mx, bad);
  hipLaunchKernelGGL(sym_group_kernel, dim3(chunks, ncomp), dim3(256), 0, s, b, comp_prob, comp_k,
                     mx, chunks, bad);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
