// Fused FP64 log-likelihood and gradient for small dimensions (step A3 with
// its row epilogue in one launch).
//
// One workgroup takes 16 points and every component: it stages
// delta_k = x - mu_k of its rows in LDS, multiplies them by P_k on the FP64
// matrix cores (16x16x4 MFMAs, each wave owning a set of 16-column blocks of
// the K x d outputs, P read straight from the L2), forms q_k = delta_k . Y_k
// per row, the family's l, and the gradient -sum_k r_k Y_k (mixture) or
// -((nu + d)/(nu + q)) Y (Student-t) through the same LDS, and writes l and
// the gradient once.  Y and the q partials never go to HBM, and the two
// launches of the GEMM + epilogue path become one: at d <= 128 the path is
// bound by latency and launch count rather than by the matrix cores.
//
// The k index of the contraction is taken in groups of 32, each lane holding
// 8 consecutive values of its A and B rows (any order of the j sum is the
// same sum in exact arithmetic; in FP64 the rounding differs from the GEMM
// path's by a few ulps).
#include <cstdlib>

#include "internal.h"
#include "mixture.h"

namespace sb {

namespace {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kMaxSlots = 6;   // 16-column blocks per wave (K * dp <= 384)

struct FusedArgs {
  Model m;
  ASrc a;                       // kind 0: rows of X (FP64), optional row map
  int64_t M;
  const int32_t *count;         // device row count (nullable -> M)
  const int32_t *outmap;        // output row of each row (nullable)
  double *logl;
  double *grad;                 // [*][ldg] (nullable)
  int64_t ldg;
  double *aux;                  // [M][K]: responsibilities / q (nullable)
  int dp;                       // d rounded up to a multiple of 32
};

// RB row blocks of 16 points per workgroup (each B value a lane loads feeds
// RB MFMAs; the launcher uses RB = 1); NS 16-column blocks per wave, every
// wave running all NS (a wave whose last slot lies past the K x dp outputs
// multiplies block 0 again and keeps nothing of it), so that the slot loops
// hold no branch and each slot's loads wait only for their own data.  FAST:
// d is a multiple of 8 and P is 16-byte aligned (the B loads below).
template <int RB, int NS, bool FAST>
__global__ __launch_bounds__(256) void fused_logl_grad_kernel(FusedArgs f) {
  constexpr int R = 16 * RB;  // points per workgroup
  static_assert(RB == 1, "the mixture row epilogue maps 16 rows onto the 256 threads");
  extern __shared__ __attribute__((aligned(16))) double lds[];
  const Model &m = f.m;
  const int d = m.d, K = m.K, dp = f.dp, nbk = dp / 16, nb = K * nbk;
  // D rows padded by 16 bytes: the 16 rows of a fragment read start on
  // different banks (a row of dp doubles is a multiple of the bank width)
  const int ld = dp + 2;
  const int64_t M = f.count ? (int64_t)(*f.count) : f.M;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  if (r0 >= M) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // LDS: D[k][i][j] = delta_k of row i (zero past d and past M), then
  // delta_k * Y_k, then the weighted Y; qs[i][k][t] the q partial of row i, component k, column
  // block t; sc[i][k] the row's gradient weights; MU[k][j] = mu_k
  double *D = lds;
  double *qs = D + (size_t)K * R * ld;
  double *sc = qs + R * K * nbk;
  double *MU = sc + R * K;  // mu_k, zero past d: [K][dp]
  const double *X = (const double *)f.a.X;
  // beta_k of the mixture row epilogue's lane k = tid % 16 (index clamped,
  // K >= 1), loaded here so that it arrives with the staging's values
  const double beta_k = m.beta[(tid & 15) < K ? (tid & 15) : 0];
  // blocks b = wave + 4 s: column block t = b / K of component k = b % K
  const int fr = lane & 15, fg = lane >> 4;
  d4v acc[RB][NS];
  int bk[NS], bn[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q][s] = d4v{0.0, 0.0, 0.0, 0.0};
    const int b = wave + 4 * s;
    bk[s] = b < nb ? b % K : 0;
    bn[s] = b < nb ? (b / K) * 16 : 0;
  }
  // k in groups of 32: in group g lane l holds the 8 consecutive values j =
  // 32 g + 8 (l / 16) + u, u < 8, of its B row (n = bn + l % 16 of P_k) and
  // of its A row, and MFMA u of the group takes them (each MFMA sums four
  // k values 8 apart; every k of the group exactly once).  A lane's B values
  // are two full 32-byte runs of one row, 16 rows per load: whole cache
  // lines.  Slot s's values of group g + 1 load as soon as its MFMAs of
  // group g have read them, so they fly while the other slots multiply.
  // With FAST a lane's 8 values lie in its row or wholly past it: the loads
  // are unconditional, from row 0 when past d, and the values are zeroed
  // where the MFMAs take them (bin), not where they land, so that no wait
  // follows the loads.
  bool bin[NS];
  auto bload = [&](int s, int g, d2v (&bv)[4]) {
    const int n = bn[s] + fr, j0 = 32 * g + 8 * fg;
    if constexpr (FAST) {
      const bool in = n < d && j0 < d;
      const double *p = m.P64 + ((size_t)bk[s] * d + (in ? n : 0)) * d + (in ? j0 : 0);
#pragma unroll
      for (int u = 0; u < 4; ++u) bv[u] = *(const d2v *)(p + 2 * u);
      bin[s] = in;
    } else {
      const double *p = m.P64 + ((size_t)bk[s] * d + n) * d + j0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool i0 = n < d && j0 + 2 * u < d, i1 = n < d && j0 + 2 * u + 1 < d;
        bv[u] = d2v{i0 ? p[2 * u] : 0.0, i1 ? p[2 * u + 1] : 0.0};
      }
      bin[s] = true;
    }
  };
  // the first k-group's P values load before the staging below, so that
  // the two round trips overlap
  d2v bb[NS][4];
#pragma unroll
  for (int s = 0; s < NS; ++s) bload(s, 0, bb[s]);

  // Staging: every global load of the tile (mu, the row map, x) is issued
  // before the first one is used, so the tile waits for one or two round
  // trips rather than one per value.  Values go in pairs (j, j + 1): a
  // thread takes at most kPairs pairs of x (R dp / 2 <= 1024 for dp <= 128)
  // and one pair of mu (K dp / 2 <= 192).
  constexpr int kPairs = 4;
  const int hp = dp / 2, np = R * hp;
  const int mk = tid < K * hp ? tid / hp : -1, mj = 2 * (tid % hp);
  double mv0 = 0.0, mv1 = 0.0;
  if (mk >= 0) {
    const double *p = m.mu64 + (size_t)mk * d + mj;
    if (mj < d) mv0 = p[0];
    if (mj + 1 < d) mv1 = p[1];
  }
  // source row of each pair (-1 past M); the map is read at a clamped row,
  // without a branch, so its loads issue together
  int64_t src[kPairs];
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    const int64_t row = r0 + (tid + 256 * u) / hp;
    src[u] = row < M ? row : M - 1;
  }
  if (f.a.rowmap) {
#pragma unroll
    for (int u = 0; u < kPairs; ++u) src[u] = f.a.rowmap[src[u]];
  }
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    const int e = tid + 256 * u;
    if (e >= np || r0 + e / hp >= M) src[u] = -1;
  }
  d2v xv[kPairs];
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    const int j = 2 * ((tid + 256 * u) % hp);
    const double *p = X + src[u] * f.a.ldx + j;
    xv[u] = d2v{src[u] >= 0 && j < d ? p[0] : 0.0, src[u] >= 0 && j + 1 < d ? p[1] : 0.0};
  }
  if (mk >= 0) *(d2v *)&MU[mk * dp + mj] = d2v{mv0, mv1};
  __syncthreads();
  // D[k][i][j] = delta_k of row i (zero past d and past M)
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    const int e = tid + 256 * u;
    if (e < np) {
      const int i = e / hp, j = 2 * (e % hp);
      for (int k = 0; k < K; ++k)
        *(d2v *)&D[((size_t)k * R + i) * ld + j] =
            src[u] >= 0 ? xv[u] - *(const d2v *)&MU[k * dp + j] : d2v{0.0, 0.0};
    }
  }
  __syncthreads();

  const int ng = dp / 32;
  for (int g = 0; g < ng; ++g) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const double *ar = &D[((size_t)bk[s] * R + 16 * q + fr) * ld + 32 * g + 8 * fg];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const d2v av = *(const d2v *)(ar + 2 * u);
          const d2v bv = bin[s] ? bb[s][u] : d2v{0.0, 0.0};
          acc[q][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], bv[0], acc[q][s], 0, 0, 0);
          acc[q][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], bv[1], acc[q][s], 0, 0, 0);
        }
      }
      if (g + 1 < ng) bload(s, g + 1, bb[s]);
    }
  }

  // q partials: item v of lane l is Y_k[row 16 q + fg + 4 v][column bn + fr];
  // once every wave is done reading D as the A operand, each item's product
  // delta_k * Y_k replaces its delta in D, and qs[i][k][t] sums block t's 16
  // products of row i in column order (threads along rows: the rows' 8-byte
  // reads fall on different banks)
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (wave + 4 * s < nb) {
#pragma unroll
      for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double *t = &D[((size_t)bk[s] * R + 16 * q + fg + 4 * v) * ld + bn[s] + fr];
          *t = *t * acc[q][s][v];
        }
    }
  }
  __syncthreads();
  for (int e = tid; e < R * K * nbk; e += 256) {
    const int i = e % R, k = (e / R) % K, t = e / (R * K);
    const double *p = &D[((size_t)k * R + i) * ld + 16 * t];
    double q = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) q += p[c];
    qs[(i * K + k) * nbk + t] = q;
  }
  __syncthreads();

  // per row: l, the responsibilities (or the Student-t weight) in FP64
  if (m.family == SB_FAMILY_STUDENT_T) {
    if (tid < R) {
      const int i = tid;
      const int64_t row = r0 + i;
      if (row < M) {
        const int64_t orow = f.outmap ? (int64_t)f.outmap[row] : row;
        const double *qp = qs + (size_t)i * K * nbk;
        double q = 0;
        for (int t = 0; t < nbk; ++t) q += qp[t];
        const double nd = m.nu + (double)d;
        f.logl[orow] = m.c + m.beta[0] - 0.5 * nd * log1p(q / m.nu);
        if (f.aux) f.aux[row * K] = q;
        sc[i * K] = nd / (m.nu + q);
      }
    }
  } else {
    // 16 lanes per row (R = 16 rows of 16 = 256 threads), component k in
    // lane k (K <= 12 here): a_k = beta_k - q_k / 2, the wave maximum, each
    // exp(a_k - max) formed once in its lane and the K of them added in
    // component order from zero, lse = max + log(sum) (a_0 when K = 1),
    // r_k = exp(a_k - lse): the arithmetic and order of the row epilogue
    // of the two-launch path
    const int i = tid >> 4, k = tid & 15, base = (tid & 63) & ~15;
    const int64_t row = r0 + i;
    double a = -INFINITY;
    if (k < K) {
      const double *qp = qs + ((size_t)i * K + k) * nbk;
      double q = 0;
      for (int t = 0; t < nbk; ++t) q += qp[t];
      a = beta_k - 0.5 * q;
    }
    double mx = a;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    double lse;
    if (K == 1) {
      lse = __shfl(a, base, 64);
    } else {
      const double e = k < K ? exp(a - mx) : 0.0;
      double ssum = 0;
      for (int c = 0; c < K; ++c) ssum += __shfl(e, base + c, 64);
      lse = mx + log(ssum);
    }
    if (row < M && k < K) {
      const double r = K == 1 ? 1.0 : exp(a - lse);
      sc[i * K + k] = r;
      if (f.aux) f.aux[row * K + k] = r;
      if (k == 0) f.logl[f.outmap ? (int64_t)f.outmap[row] : row] = m.c + lse;
    }
  }
  if (!f.grad) return;
  __syncthreads();  // (also: every wave is done reading D)
  // D <- weight_k * Y_k (a component of weight zero adds nothing, as in the
  // two-launch path)
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (wave + 4 * s < nb) {
#pragma unroll
      for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * q + fg + 4 * v;
          const double w = sc[i * K + bk[s]];
          D[((size_t)bk[s] * R + i) * ld + bn[s] + fr] = w != 0.0 ? w * acc[q][s][v] : 0.0;
        }
    }
  }
  __syncthreads();
  // grad = -sum_k D_k, components in order, 16-byte stores where aligned
  for (int e = tid; e < R * (dp / 2); e += 256) {
    const int i = e / (dp / 2), j = 2 * (e % (dp / 2));
    const int64_t row = r0 + i;
    if (row >= M || j >= d) continue;
    d2v s = d2v{0.0, 0.0};
    for (int k = 0; k < K; ++k) s += *(const d2v *)&D[((size_t)k * R + i) * ld + j];
    const int64_t orow = f.outmap ? (int64_t)f.outmap[row] : row;
    double *go = f.grad + orow * f.ldg + j;
    if (j + 1 < d && (((uintptr_t)go) & 15) == 0) {
      *(d2v *)go = -s;
    } else {
      go[0] = -s[0];
      if (j + 1 < d) go[1] = -s[1];
    }
  }
}

template <int NS>
void launch_fused(bool fast, dim3 grid, size_t lds, hipStream_t s, const FusedArgs &f) {
  if (fast)
    hipLaunchKernelGGL((fused_logl_grad_kernel<1, NS, true>), grid, dim3(256), lds, s, f);
  else
    hipLaunchKernelGGL((fused_logl_grad_kernel<1, NS, false>), grid, dim3(256), lds, s, f);
}

}  // namespace

bool fused_logl_grad_ok(const Model &m, const ASrc &a) {
  const char *e = getenv("SB_FUSED");  // "0": the two-launch path (for comparison)
  if (e && e[0] == '0') return false;
  // d <= 128: there one launch beats the GEMM + epilogue pair (c1, d = 64,
  // K = 4: 18.3 vs 13.3 + 7.4 us); at d = 256 (c2) the 64 x 64-tile GEMM's
  // staged P outruns the fused kernel's P stream (36.6 + 8.6 vs 48.5 us)
  const int dp = (m.d + 31) / 32 * 32;
  return a.kind == 0 && !a.zero_mu && m.d >= 1 && dp <= 128 && m.K >= 1 && m.K <= kMaxK &&
         (int64_t)m.K * dp <= 16 * 4 * kMaxSlots && m.P64 && m.mu64 &&
         (m.family == SB_FAMILY_GAUSS_MIX || (m.family == SB_FAMILY_STUDENT_T && m.K == 1));
}

int launch_fused_logl_grad(const Model &m, const ASrc &a, int64_t M, const int32_t *count,
                           const int32_t *outmap, double *logl, double *grad, int64_t ldg,
                           double *aux, hipStream_t s) {
  if (!fused_logl_grad_ok(m, a)) {
    set_error("fused logL+grad: unsupported model or operand");
    return SB_E_UNSUPPORTED;
  }
  if (M <= 0) return SB_OK;
  FusedArgs f;
  f.m = m;
  f.a = a;
  f.M = M;
  f.count = count;
  f.outmap = outmap;
  f.logl = logl;
  f.grad = grad;
  f.ldg = ldg;
  f.aux = aux;
  f.dp = (m.d + 31) / 32 * 32;
  const int nbk = f.dp / 16;
  // one row block of 16 points per workgroup: two (32 points) measured slower
  // at c1 and c2 (one wave per SIMD at 290 registers) and would take more
  // than 64 KB of LDS there
  constexpr int R = 16;
  const size_t lds =
      8 * ((size_t)m.K * R * (f.dp + 2) + (size_t)R * m.K * nbk + (size_t)R * m.K +
           (size_t)m.K * f.dp);
  const dim3 grid((unsigned)ceil_div(M, R));
  const bool fast = m.d % 8 == 0 && (((uintptr_t)m.P64) & 15) == 0;
  switch ((m.K * nbk + 3) / 4) {  // 16-column blocks per wave
    case 1: launch_fused<1>(fast, grid, lds, s, f); break;
    case 2: launch_fused<2>(fast, grid, lds, s, f); break;
    case 3: launch_fused<3>(fast, grid, lds, s, f); break;
    case 4: launch_fused<4>(fast, grid, lds, s, f); break;
    case 5: launch_fused<5>(fast, grid, lds, s, f); break;
    default: launch_fused<6>(fast, grid, lds, s, f); break;
  }
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
