// BF16 matrix-core contraction of step A3 for d a multiple of 8:
//   Y_k = (X - mu_k) P_k^T,  q_k = sum_n (X - mu_k)_n Y_kn   (FP32 accumulation)
// NPROD = 1: BF16 operands (the mixed-precision discovery GEMM).
// NPROD = 3: FP32 data as split operands v = hi + lo, hi = bf16(v),
//   lo = bf16(v - hi); the product is hi*hi + hi*lo + lo*hi (lo*lo, ~2^-16
//   relative, is dropped), so one FP32-accurate-to-~2^-16 contraction costs
//   three BF16 MFMAs instead of eight FP32 ones.
// Tile: 128 x 128 outputs per workgroup (four waves of 64 x 64, each a 4 x 4
// grid of 16x16x32 MFMAs), k-tiles staged through LDS, the next k-tile
// prefetched into registers while the current one is multiplied.
#include <algorithm>

#include "internal.h"

namespace sb {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));

struct Bf16Params {
  ASrc a;                   // points: rows of X (kind 0) or ray points (kind 1), FP32
  int64_t M;
  const int32_t *count;     // device row count (nullable -> M)
  int d, K, ntn;
  const float *mu;          // [K][d]
  const bf16_t *Phi, *Plo;  // [K][d][d]
  float *Y;                 // [M][ldy] (nullable)
  int64_t ldy;
  float *qpart;             // [M][K][ntn]
};

typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

// Two FP32 values to packed BF16, round to nearest even (one v_cvt_pk_bf16_f32).
__device__ inline uint32_t pack2(float a, float b) {
  const bf2v h = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, h);
}
// The FP32 values of a packed pair (low half, high half).
__device__ inline float lo_half(uint32_t u) { return __builtin_bit_cast(float, u << 16); }
__device__ inline float hi_half(uint32_t u) { return __builtin_bit_cast(float, u & 0xffff0000u); }

// Launch bounds: workgroup size and the minimum waves per SIMD the register
// allocation must leave room for.
template <int BM, int BN, int BK, int KIND, int NPROD, int NT>
struct Bf16Occ {
  static constexpr int value =
      NT == 512 ? 2
                : ((BM == 128 && BN == 128) ? ((BK == 32 && !(KIND == 1 && NPROD == 3)) ? 3 : 2) : 1);
};

// NT = 64 * WGM * WGN threads: a WGM x WGN grid of waves, each owning a
// (BM / WGM) x (BN / WGN) block of the tile.
template <int NPROD, int KIND, int BM, int BN, int BK, int WGM = 2, int WGN = 2>
__global__ __launch_bounds__(64 * WGM * WGN, (Bf16Occ<BM, BN, BK, KIND, NPROD, 64 * WGM * WGN>::value))
void quad_gemm_bf16_kernel(Bf16Params g) {
  constexpr int NT = 64 * WGM * WGN;
  // LDS rows of BK bf16 without padding; the 16-byte chunk c of row r sits
  // at chunk c ^ swz(r), swz(r) = (r / R) mod C (C chunks per row, R rows per
  // 32 banks): the row-wise tile stores and the 8-row fragment reads both
  // touch 32 distinct banks per cycle.
  constexpr int C = BK / 8, R = 64 / BK;
  auto lds = [](int row, int kel) {  // element index of (row, k) in an LDS tile
    return row * BK + ((((kel >> 3) ^ ((row / R) % C))) << 3) + (kel & 7);
  };
  constexpr int WM = BM / WGM, TM = WM / 16;  // wave tile WM x WN: TM x TN MFMA blocks
  constexpr int WN = BN / WGN, TN = WN / 16;
  constexpr int VA = BK / 4;          // float4 per A row per k-tile
  constexpr int NA = BM * VA / NT;    // float4 loads per thread
  constexpr int VB = BK / 8;          // 8-bf16 vectors per B row per k-tile
  constexpr int NB = BN * VB / NT;    // per thread and operand half
  constexpr bool SPLIT = NPROD == 3;
  static_assert(NA >= 1 && NB >= 1 && NT % VA == 0 && NT % VB == 0, "tile");
  __shared__ __attribute__((aligned(16))) bf16_t Ah[BM * BK];
  __shared__ __attribute__((aligned(16))) bf16_t Al[SPLIT ? BM * BK : 8];
  __shared__ __attribute__((aligned(16))) bf16_t Bh[BN * BK];
  __shared__ __attribute__((aligned(16))) bf16_t Bl[SPLIT ? BN * BK : 8];
  __shared__ float qs[WGN][BM];

  // XCD-aware tile order.  Workgroup w runs on XCD w % 8; each XCD owns a
  // fixed set of column blocks (component k, n-tile) and walks the M-tiles
  // in order, so the workgroups sharing an M-tile's rows of A run together
  // on one L2 and the XCD's column blocks of P stay resident in it.
  const int ncol = g.K * g.ntn;
  const int64_t w = blockIdx.x;
  int col;
  int64_t mt;
  if (ncol % 8 == 0) {
    const int per = ncol / 8;
    const int64_t li = w / 8;
    col = (int)(w % 8) + 8 * (int)(li % per);
    mt = li / per;
  } else {
    col = (int)(w % ncol);
    mt = w / ncol;
  }
  const int64_t M = g.count ? (int64_t)(*g.count) : g.M;
  const int64_t m0 = mt * BM;
  if (m0 >= M) return;
  const int d = g.d;
  const int k = col / g.ntn, nt = col % g.ntn;
  const int n0 = nt * BN;
  const float *mu = g.mu + (size_t)k * d;
  const char *Phb = (const char *)(g.Phi + (size_t)k * d * d);
  const char *Plb = SPLIT ? (const char *)(g.Plo + (size_t)k * d * d) : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  // Element offset of point row `row`'s data (kind 0: its X row; kind 1: its
  // ray's endpoint rows) and the ray parameter t.  The host guarantees the
  // operand arrays are below 4 GiB, so byte offsets fit in 32 bits.
  auto row_off = [&](int64_t row, uint32_t &off, float &t) {
    if constexpr (KIND == 0) {
      const int64_t r = g.a.rowmap ? (int64_t)g.a.rowmap[row] : row;
      off = (uint32_t)(r * g.a.ldx);
      t = 0.f;
    } else {
      const int64_t ray = row / g.a.n_pts;
      const int jj = (int)(row % g.a.n_pts);
      t = ((float)jj + 0.5f) / (float)g.a.n_pts;
      off = (uint32_t)(ray * d);
    }
  };
  const char *Xa = (const char *)(KIND == 0 ? g.a.X : g.a.P0);
  const char *Xb = (const char *)g.a.P1;
  const int ca = tid % VA, cb = tid % VB;
  uint32_t aoff[NA];  // byte offsets of this thread's A rows (rows >= M read row m0)
  float tpar[NA];
  bool aok[NA];
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    const int64_t row = m0 + (tid + NT * r) / VA;
    aok[r] = row < M;
    uint32_t off;
    row_off(aok[r] ? row : m0, off, tpar[r]);
    aoff[r] = 4u * (off + (uint32_t)(ca * 4));
  }
  uint32_t boff[NB];  // byte offsets of this thread's B rows (rows >= d read row 0)
  bool bok[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    const int n = n0 + (tid + NT * r) / VB;
    bok[r] = n < d;
    boff[r] = 2u * ((uint32_t)(bok[r] ? n : 0) * (uint32_t)d + (uint32_t)(cb * 8));
  }
  const uint32_t muoff = 4u * (uint32_t)(ca * 4);

  f4v ra[NA], rq[NA], rmu;
  u4v rbh[NB], rbl[NB];
  // k-tile loads.  Rows past M (A) or d (B) read a clamped valid row: they
  // feed only outputs that are never written.  A whole k-tile (the uniform
  // case k0 + BK <= d) loads unconditionally; the tail zeroes k >= d.
  auto load = [&](int k0) {
    const uint32_t ka = 4u * (uint32_t)k0, kb = 2u * (uint32_t)k0;
    if (k0 + BK <= d) {
#pragma unroll
      for (int r = 0; r < NA; ++r) {
        ra[r] = *(const f4v *)(Xa + (aoff[r] + ka));
        if constexpr (KIND == 1) rq[r] = *(const f4v *)(Xb + (aoff[r] + ka));
      }
      rmu = *(const f4v *)((const char *)mu + (muoff + ka));
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        rbh[r] = *(const u4v *)(Phb + (boff[r] + kb));
        if constexpr (SPLIT) rbl[r] = *(const u4v *)(Plb + (boff[r] + kb));
      }
    } else {
      const bool kin = k0 + ca * 4 < d;
#pragma unroll
      for (int r = 0; r < NA; ++r) {
        ra[r] = kin ? *(const f4v *)(Xa + (aoff[r] + ka)) : f4v{0.f, 0.f, 0.f, 0.f};
        if constexpr (KIND == 1)
          rq[r] = kin ? *(const f4v *)(Xb + (aoff[r] + ka)) : f4v{0.f, 0.f, 0.f, 0.f};
      }
      rmu = kin ? *(const f4v *)((const char *)mu + (muoff + ka)) : f4v{0.f, 0.f, 0.f, 0.f};
      const bool kbin = k0 + cb * 8 < d;
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        rbh[r] = kbin ? *(const u4v *)(Phb + (boff[r] + kb)) : u4v{0u, 0u, 0u, 0u};
        if constexpr (SPLIT) rbl[r] = kbin ? *(const u4v *)(Plb + (boff[r] + kb)) : u4v{0u, 0u, 0u, 0u};
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      const int i = (tid + NT * r) / VA;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float x;
        if constexpr (KIND == 0) {
          x = ra[r][e];
        } else {
#pragma clang fp contract(off)
          x = ra[r][e] + tpar[r] * (rq[r][e] - ra[r][e]);
        }
        v[e] = x - rmu[e];  // k >= d: both zero
      }
      const uint32_t h01 = pack2(v[0], v[1]), h23 = pack2(v[2], v[3]);
      const int ai = lds(i, ca * 4);
      *(u2v *)&Ah[ai] = u2v{h01, h23};
      if constexpr (SPLIT) {
        // v - hi is exact in FP32 (hi holds v's leading bits); lo rounds it
        const uint32_t l01 = pack2(v[0] - lo_half(h01), v[1] - hi_half(h01));
        const uint32_t l23 = pack2(v[2] - lo_half(h23), v[3] - hi_half(h23));
        *(u2v *)&Al[ai] = u2v{l01, l23};
      }
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int n = (tid + NT * r) / VB;
      const int bi = lds(n, cb * 8);
      *(u4v *)&Bh[bi] = rbh[r];
      if constexpr (SPLIT) *(u4v *)&Bl[bi] = rbl[r];
    }
  };

  f4v acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  const int fr = lane & 15, fk = 8 * (lane >> 4);
  load(0);
  for (int k0 = 0; k0 < d; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < d) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      // B fragments of this k-step, then one A row block at a time: only
      // two A fragments are live, and TN independent MFMAs separate two
      // updates of one accumulator (small cross terms first)
      bf8v bhv[TN], blv[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = lds(wn * WN + j * 16 + fr, kk + fk);
        bhv[j] = *(const bf8v *)&Bh[o];
        if constexpr (SPLIT) blv[j] = *(const bf8v *)&Bl[o];
      }
      // A fragments of row block i + 1 are read while block i multiplies
      bf8v ahb[2], alb[2];
      {
        const int o = lds(wm * WM + fr, kk + fk);
        ahb[0] = *(const bf8v *)&Ah[o];
        if constexpr (SPLIT) alb[0] = *(const bf8v *)&Al[o];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int cbuf = i & 1;
        if (i + 1 < TM) {
          const int o = lds(wm * WM + (i + 1) * 16 + fr, kk + fk);
          ahb[cbuf ^ 1] = *(const bf8v *)&Ah[o];
          if constexpr (SPLIT) alb[cbuf ^ 1] = *(const bf8v *)&Al[o];
        }
        const bf8v ah = ahb[cbuf];
        if constexpr (SPLIT) {
          const bf8v al = alb[cbuf];
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bhv[j], acc[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, blv[j], acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bhv[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // Epilogue: Y, and per-row partial q over this tile's columns.  Item v of
  // lane l holds row 4 (l / 16) + v, column l % 16 of its 16 x 16 block.
  const int lr = lane >> 4, lc = lane & 15;
  float qrow[TM][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) qrow[i][v] = 0.f;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = m0 + wm * WM + i * 16 + 4 * lr + v;
      if (row >= M) continue;
      uint32_t off;
      float tt;
      row_off(row, off, tt);
      const float *pa = (const float *)Xa + off;
      const float *pb = (const float *)Xb + off;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = n0 + wn * WN + j * 16 + lc;
        if (n >= d) continue;
        const float yv = acc[i][j][v];
        if (g.Y) g.Y[row * g.ldy + (int64_t)k * d + n] = yv;
        float x;
        if constexpr (KIND == 0) {
          x = pa[n];
        } else {
#pragma clang fp contract(off)
          x = pa[n] + tt * (pb[n] - pa[n]);
        }
        qrow[i][v] += (x - mu[n]) * yv;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float t = qrow[i][v];
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
      for (int v = 0; v < 4; ++v) qs[wn][wm * WM + i * 16 + 4 * lr + v] = qrow[i][v];
  }
  __syncthreads();
  if (g.qpart) {
    for (int i = tid; i < BM; i += NT) {
      const int64_t row = m0 + i;
      if (row < M) {
        float q = qs[0][i];
#pragma unroll
        for (int w2 = 1; w2 < WGN; ++w2) q += qs[w2][i];
        g.qpart[(row * g.K + k) * g.ntn + nt] = q;
      }
    }
  }
}

// hi = bf16(fp32(x)), lo = bf16(fp32(x - hi)) for n values.
__global__ void split_bf16_kernel(int64_t n, const double *x, bf16_t *hi, bf16_t *lo) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const bf16_t h = f32_to_bf16((float)x[i]);
    hi[i] = h;
    if (lo) lo[i] = f32_to_bf16((float)(x[i] - (double)bf16_to_f32(h)));
  }
}

}  // namespace

bool quad_gemm_bf16_ok(int d) { return d >= 8 && d % 8 == 0; }

int launch_quad_gemm_bf16(int nprod, const Model &m, const ASrc &a, int64_t M,
                          const int32_t *count, QuadOut &o, hipStream_t s, TileCfg t) {
  if (!quad_gemm_bf16_ok(m.d)) {
    set_error("BF16 contraction needs d a multiple of 8 (got %d)", m.d);
    return SB_E_UNSUPPORTED;
  }
  if (!m.mu32 || !m.Phi || (nprod == 3 && !m.Plo) || a.zero_mu) {
    set_error("BF16 model copies missing");
    return SB_E_INVAL;
  }
  // operand arrays addressed with 32-bit byte offsets
  const int64_t a_rows = a.kind == 0 ? std::max<int64_t>(a.rows, M) : ceil_div(M, a.n_pts);
  const int64_t a_ld = a.kind == 0 ? a.ldx : m.d;
  if (4 * a_rows * a_ld >= ((int64_t)1 << 32) || 2 * (int64_t)m.d * m.d >= ((int64_t)1 << 32)) {
    set_error("BF16 contraction operands above 4 GiB");
    return SB_E_UNSUPPORTED;
  }
  // variants (BM, BN, BK); ray points take the 32-wide k-tile (register budget)
  int BM = (t.bm == 256) ? 256 : 128;
  int BN = (t.bn == 256) ? 256 : 128;  // 256 x 256 runs on 8 waves (2 x 4)
  int BK = (t.bk == 64 && a.kind == 0 && BN == 128 && BM == 128) ? 64 : 32;
  if (a.kind == 1 && BN == 128) BM = 128;
  Bf16Params p;
  p.a = a;
  p.M = M;
  p.count = count;
  p.d = m.d;
  p.K = m.K;
  p.ntn = (int)ceil_div(m.d, BN);
  p.mu = m.mu32;
  p.Phi = m.Phi;
  p.Plo = m.Plo;
  p.Y = (float *)o.Y;
  p.ldy = o.ldy;
  p.qpart = (float *)o.qpart;
  o.ntn = p.ntn;
  const int64_t ntile = ceil_div(M, BM) * (int64_t)(m.K * p.ntn);
  if (ntile == 0) return SB_OK;
  if (ntile > 0x7fffffffll) {
    set_error("contraction too large for one launch (%lld tiles)", (long long)ntile);
    return SB_E_UNSUPPORTED;
  }
  dim3 grid((unsigned)ntile);
#define SB_BF(NP, KD, BMv, BNv, BKv) \
  hipLaunchKernelGGL((quad_gemm_bf16_kernel<NP, KD, BMv, BNv, BKv>), grid, dim3(256), 0, s, p)
#define SB_BF8(NP, KD) \
  hipLaunchKernelGGL((quad_gemm_bf16_kernel<NP, KD, 256, 256, 32, 2, 4>), grid, dim3(512), 0, s, p)
  if (a.kind == 1 && BM == 256 && BN == 256) {
    if (nprod == 3) SB_BF8(3, 1);
    else SB_BF8(1, 1);
  } else if (a.kind == 1) {
    if (nprod == 3 && BN == 128) SB_BF(3, 1, 128, 128, 32);
    else if (nprod == 3) SB_BF(3, 1, 128, 256, 32);
    else if (BN == 128) SB_BF(1, 1, 128, 128, 32);
    else SB_BF(1, 1, 128, 256, 32);
  } else if (BM == 256 && BN == 256) {
    if (nprod == 3) SB_BF8(3, 0);
    else SB_BF8(1, 0);
  } else if (nprod == 3) {
    if (BM == 128 && BN == 128 && BK == 32) SB_BF(3, 0, 128, 128, 32);
    else if (BM == 128 && BN == 128) SB_BF(3, 0, 128, 128, 64);
    else if (BM == 256 && BN == 128) SB_BF(3, 0, 256, 128, 32);
    else SB_BF(3, 0, 128, 256, 32);
  } else {
    if (BM == 128 && BN == 128 && BK == 32) SB_BF(1, 0, 128, 128, 32);
    else if (BM == 128 && BN == 128) SB_BF(1, 0, 128, 128, 64);
    else if (BM == 256 && BN == 128) SB_BF(1, 0, 256, 128, 32);
    else SB_BF(1, 0, 128, 256, 32);
  }
#undef SB_BF8
#undef SB_BF
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int launch_split_bf16(int64_t n, const double *x, bf16_t *hi, bf16_t *lo, hipStream_t s) {
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(split_bf16_kernel, dim3((unsigned)std::min<int64_t>(8192, ceil_div(n, 256))),
                     dim3(256), 0, s, n, x, hi, lo);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
