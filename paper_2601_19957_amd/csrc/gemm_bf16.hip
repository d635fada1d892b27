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
  float *qpart;             // [M][K][ntn] (nullable)
  // Sum-of-squares mode: B holds U_k = L_k^T (upper triangular, P_k = L_k L_k^T),
  // the k-loop starts at the column tile's first column (U's rows below it
  // are zero there) and qpart gets sum_n Z_n^2 of Z = (X - mu_k) U_k^T; no Y.
  int sumsq;
  const int32_t *ymap;      // Y row of GEMM row r: ymap[r] (nullable: r)
  int64_t ycol;             // column offset of the Y block
  int yneg;                 // store -Y (q still uses Y)
  // Grouped by component (nullable): component k multiplies gcnt[k] rows,
  // listed at a.rowmap + k * gcap (X rows) and ymap + k * gcap (Y rows);
  // qpart is then indexed by the Y row
  const int32_t *gcnt;
  int64_t gcap;
  // grouped: gradient rows of the rows with a single listed component, -Y
  // into them instead of Y (QuadOut::gdst)
  const int32_t *gdst;
  float *gdir;
  int64_t ldg;
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

// Rows per epilogue pass: the largest WM / 2^i (at least 16) within `fit`.
constexpr int stage_rows(int wm, int fit) {
  int r = wm;
  while (r > 16 && r > fit) r /= 2;
  return r;
}

// Launch bounds: workgroup size and the minimum waves per SIMD the register
// allocation must leave room for.
template <int BM, int BN, int BK, int KIND, int NPROD, int NT, int NS>
struct Bf16Occ {
  static constexpr int value =
      (NT == 512 || NS == 2)
          ? 2
          : ((BM == 128 && BN == 128) ? ((BK == 32 && !(KIND == 1 && NPROD == 3)) ? 3 : 2) : 1);
};

// One output tile (w: the tile's index in the launch's tile order).
// NT = 64 * WGM * WGN threads: a WGM x WGN grid of waves, each owning a
// (BM / WGM) x (BN / WGN) block of the tile.  NS LDS stages: with one, a
// k-tile is stored, multiplied and released between two barriers; with two
// (ping-pong), the split and store of k-tile t + 1 run beside the MFMAs of
// k-tile t, one barrier per k-tile.
template <int NPROD, int KIND, int BM, int BN, int BK, int WGM, int WGN, int NS>
__device__ __forceinline__ void bf16_tile(const Bf16Params &g, const int64_t w, const int tid) {
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
  static_assert(NS == 1 || NS == 2, "stages");
  // One LDS arena: the k-tile stages during the main loop, then the
  // epilogue's per-wave staging of the accumulators (SR rows of WN + 4
  // floats per wave and pass).
  constexpr int NH = SPLIT ? 2 : 1;  // operand halves
  constexpr int MAIN_B = NS * NH * (BM + BN) * BK * 2;
  constexpr int NWV = WGM * WGN, SLD = WN + 4;
  // LDS a workgroup may take without lowering its occupancy (known for the
  // square tiles, whose register use meets the launch bound); the staging
  // may grow the arena up to it
  constexpr int WGCU = (Bf16Occ<BM, BN, BK, KIND, NPROD, NT, NS>::value * 4) / NWV;
  constexpr int CAP = BM == BN ? (160 * 1024) / (WGCU > 0 ? WGCU : 1) - WGN * BM * 4 - 1024 : 0;
  constexpr int SR = stage_rows(WM, (MAIN_B > CAP ? MAIN_B : CAP) / (NWV * SLD * 4));
  constexpr int ARENA_B = MAIN_B > NWV * SR * SLD * 4 ? MAIN_B : NWV * SR * SLD * 4;
  static_assert(WM % SR == 0, "epilogue passes");
  __shared__ __attribute__((aligned(16))) char arena[ARENA_B];
  bf16_t *const Ah = (bf16_t *)arena;
  bf16_t *const Al = Ah + NS * BM * BK;
  bf16_t *const Bh = Ah + NH * NS * BM * BK;
  bf16_t *const Bl = Bh + NS * BN * BK;
  __shared__ float qs[WGN][BM];

  // XCD-aware tile order.  Workgroup w runs on XCD w % 8; each XCD owns a
  // fixed set of column blocks (component k, n-tile) and walks the M-tiles
  // in order, so the workgroups sharing an M-tile's rows of A run together
  // on one L2 and the XCD's column blocks of P stay resident in it.
  const int ncol = g.K * g.ntn;
  int col = 0;
  int64_t mt = 0, M;
  const int32_t *rmap = g.a.rowmap, *ymp = g.ymap, *gdp = nullptr;
  if (g.gcnt) {
    // row tiles of the components one after another (ceil(gcnt[k] / BM) each,
    // a count above the lists' capacity taken as the capacity), each row tile
    // followed by its ntn column tiles: T tiles in all.  The grid is a
    // multiple of 8 and at least T; XCD x takes tiles [x c, (x + 1) c),
    // c = ceil(T / 8), in order, so the column tiles of a row tile (which
    // read the same rows of X) run together on one L2.
    auto cnt = [&](int q) { return (int64_t)min((int64_t)g.gcnt[q], g.gcap); };
    int64_t nrt = 0;
    for (int q = 0; q < g.K; ++q) nrt += (cnt(q) + BM - 1) / BM;
    const int64_t per = (nrt * g.ntn + 7) / 8, li = w / 8;
    if (li >= per) return;
    const int64_t t = (w % 8) * per + li;
    if (t >= nrt * g.ntn) return;
    const int64_t tt = t / g.ntn;
    int kk = -1;
    int64_t acc = 0;
    for (int q = 0; q < g.K; ++q) {
      const int64_t nq = (cnt(q) + BM - 1) / BM;
      if (kk < 0 && tt < acc + nq) {
        kk = q;
        mt = tt - acc;
      }
      acc += nq;
    }
    if (kk < 0) return;
    col = kk * g.ntn + (int)(t % g.ntn);
    M = cnt(kk);
    rmap += (int64_t)kk * g.gcap;
    ymp += (int64_t)kk * g.gcap;
    if (g.gdst) gdp = g.gdst + (int64_t)kk * g.gcap;
  } else {
    if (ncol % 8 == 0) {
      const int per = ncol / 8;
      const int64_t li = w / 8;
      col = (int)(w % 8) + 8 * (int)(li % per);
      mt = li / per;
      if (g.sumsq) {
        // the triangle makes column tile nt cost (d - nt BN): rotate each
        // component's tiles by its first column's slot so every XCD gets a
        // mix of long and short tiles (a bijection within each component)
        const int kc = col / g.ntn;
        col = kc * g.ntn + (col % g.ntn + (kc * g.ntn) / 8) % g.ntn;
      }
    } else {
      col = (int)(w % ncol);
      mt = w / ncol;
    }
    M = g.count ? (int64_t)(*g.count) : g.M;
  }
  const int64_t m0 = mt * BM;
  if (m0 >= M) return;
  const int d = g.d;
  const int k = col / g.ntn, nt = col % g.ntn;
  const int n0 = nt * BN;
  const float *mu = g.mu + (size_t)k * d;
  const char *Phb = (const char *)(g.Phi + (size_t)k * d * d);
  const char *Plb = SPLIT ? (const char *)(g.Plo + (size_t)k * d * d) : nullptr;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  // Element offset of point row `row`'s data (kind 0: its X row; kind 1: its
  // ray's endpoint rows) and the ray parameter t.  The host guarantees the
  // operand arrays are below 4 GiB, so byte offsets fit in 32 bits.
  auto row_off = [&](int64_t row, uint32_t &off, float &t) {
    if constexpr (KIND == 0) {
      const int64_t r = rmap ? (int64_t)rmap[row] : row;
      off = (uint32_t)(r * g.a.ldx);
      t = 0.f;
    } else {
      const int64_t ray = row / g.a.n_pts;
      const int jj = (int)(row % g.a.n_pts);
      t = g.a.dt > 0.f ? g.a.t0 + (float)jj * g.a.dt : ((float)jj + 0.5f) / (float)g.a.n_pts;
      off = (uint32_t)(ray * d);
    }
  };
  const char *Xa = (const char *)(KIND == 0 ? g.a.X : g.a.P0);
  const char *Xb = (const char *)g.a.P1;
  const int ca = tid % VA, cb = tid % VB;
  // This thread's A rows within the tile: rows of X are spread over the
  // workgroup (one row per VA threads and load); ray points take NA
  // consecutive rows, so when NA divides the points per ray they lie on one
  // ray and share one load of each endpoint chunk.
  auto arow = [&](int r) { return KIND == 1 ? (tid / VA) * NA + r : (tid + NT * r) / VA; };
  const bool one_ray = KIND == 1 && g.a.n_pts % NA == 0;
  uint32_t aoff[NA];  // byte offsets of this thread's A rows (rows >= M read row m0)
  float tpar[NA];
  bool aok[NA];
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    const int64_t row = m0 + arow(r);
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
      if (one_ray) {
        const f4v p0 = *(const f4v *)(Xa + (aoff[0] + ka)), p1 = *(const f4v *)(Xb + (aoff[0] + ka));
#pragma unroll
        for (int r = 0; r < NA; ++r) {
          ra[r] = p0;
          rq[r] = p1;
        }
      } else {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
          ra[r] = *(const f4v *)(Xa + (aoff[r] + ka));
          if constexpr (KIND == 1) rq[r] = *(const f4v *)(Xb + (aoff[r] + ka));
        }
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
  auto store = [&](int st) {  // into LDS stage st
    const int sa = st * BM * BK, sbo = st * BN * BK;
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      const int i = arow(r);
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
      const int ai = sa + lds(i, ca * 4);
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
      const int bi = sbo + lds(n, cb * 8);
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
  // MFMAs of the k-tile in LDS stage st
  auto mma = [&](int st) {
    const int sa = st * BM * BK, sbo = st * BN * BK;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      // B fragments of this k-step, then one A row block at a time: only
      // two A fragments are live, and TN independent MFMAs separate two
      // updates of one accumulator (small cross terms first)
      bf8v bhv[TN], blv[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = sbo + lds(wn * WN + j * 16 + fr, kk + fk);
        bhv[j] = *(const bf8v *)&Bh[o];
        if constexpr (SPLIT) blv[j] = *(const bf8v *)&Bl[o];
      }
      // A fragments of row block i + 1 are read while block i multiplies
      bf8v ahb[2], alb[2];
      {
        const int o = sa + lds(wm * WM + fr, kk + fk);
        ahb[0] = *(const bf8v *)&Ah[o];
        if constexpr (SPLIT) alb[0] = *(const bf8v *)&Al[o];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int cbuf = i & 1;
        if (i + 1 < TM) {
          const int o = sa + lds(wm * WM + (i + 1) * 16 + fr, kk + fk);
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
  };
  const int kbeg = g.sumsq ? (n0 / BK) * BK : 0;
  load(kbeg);
  if constexpr (NS == 1) {
    for (int k0 = kbeg; k0 < d; k0 += BK) {
      store(0);
      __syncthreads();
      if (k0 + BK < d) load(k0 + BK);
      mma(0);
      __syncthreads();
    }
  } else {
    // k-tile t sits in stage t & 1.  On entry to iteration t the registers
    // hold k-tile t + 1; its split and store into the other stage, and then
    // the loads of k-tile t + 2, may come before or after the MFMAs of k-tile
    // t (between two barriers nothing else touches the other stage)
    store(0);
    __syncthreads();
    const int nk = (d + BK - 1) / BK;
    int t = kbeg / BK;
    if (t + 1 < nk) load((t + 1) * BK);
    int st = 0;
    for (; t < nk; ++t) {
      const bool more = t + 1 < nk;
      mma(st);
      if (more) {
        store(st ^ 1);
        if (t + 2 < nk) load((t + 2) * BK);
        __syncthreads();
      }
      st ^= 1;
    }
  }

  const int lr = lane >> 4, lc = lane & 15;
  if (g.sumsq) {
    // q partial = sum of the squares over this tile's columns below d: item
    // v of lane l holds row 4 (l / 16) + v, column l % 16 of its 16 x 16 block
    float qrow[TM][4];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if (n0 + wn * WN + j * 16 + lc < d) t += acc[i][j][v] * acc[i][j][v];
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
  } else {
  // Epilogue.  Item v of lane l holds row 4 (l / 16) + v, column l % 16 of
  // its 16 x 16 block; each wave stages SR rows of its tile at a time in
  // LDS and writes them back as 16-byte row chunks (Y), with the partial
  // q over its columns from the same chunks of X and mu.  Passes are as
  // large as the LDS the occupancy leaves allows, so the X loads of a pass
  // are issued together.  Without qpart only Y is written.
  const bool wq = g.qpart != nullptr;
  constexpr int CPR = WN / 4, RPI = 64 / CPR;  // float4 chunks per row, rows per instruction
  constexpr int NU = SR / RPI;                 // rows per lane and pass
  static_assert(CPR <= 64 && 64 % CPR == 0 && SR % RPI == 0, "epilogue layout");
  const int er = lane / CPR, ec = lane % CPR;
  const int c0 = n0 + wn * WN + 4 * ec;  // this lane's first column
  const bool cin = c0 < d;               // d % 8 == 0: the whole chunk is in or out
  const f4v muv = cin ? *(const f4v *)(mu + c0) : f4v{0.f, 0.f, 0.f, 0.f};
  if constexpr (NS == 2) __syncthreads();  // (one stage is still being read)
  float *const stg = (float *)arena + wave * SR * SLD;
#pragma unroll
  for (int p0 = 0; p0 < WM; p0 += SR) {
#pragma unroll
    for (int i = p0 / 16; i < (p0 + SR) / 16; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) stg[(i * 16 - p0 + 4 * lr + v) * SLD + j * 16 + lc] = acc[i][j][v];
    // the wave reads back what its other lanes wrote
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int lrow = wm * WM + p0 + u * RPI + er;  // row within the tile
      const int64_t row = m0 + lrow;
      const f4v y = *(const f4v *)&stg[(u * RPI + er) * SLD + 4 * ec];
      float q = 0.f;
      if (row < M && cin) {
        if (g.Y) {
          const int64_t yrow = ymp ? (int64_t)ymp[row] : row;
          const int32_t grow = gdp ? gdp[row] : -1;
          if (grow >= 0) {
            *(f4v *)&g.gdir[(int64_t)grow * g.ldg + c0] = -y;
          } else {
            *(f4v *)&g.Y[yrow * g.ldy + g.ycol + (int64_t)k * d + c0] = g.yneg ? -y : y;
          }
        }
      }
      if (wq && row < M && cin) {
        uint32_t off;
        float tt;
        row_off(row, off, tt);
        f4v x = *(const f4v *)((const float *)Xa + off + c0);
        if constexpr (KIND == 1) {
#pragma clang fp contract(off)
          const f4v xq = *(const f4v *)((const float *)Xb + off + c0);
          for (int e = 0; e < 4; ++e) x[e] = x[e] + tt * (xq[e] - x[e]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) q += (x[e] - muv[e]) * y[e];
      }
#pragma unroll
      for (int o = 1; o < CPR; o <<= 1) q += __shfl_xor(q, o, 64);
      if (ec == 0) qs[wn][lrow] = q;
    }
    // the next pass overwrites the staging rows
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  }
  __syncthreads();
  if (g.qpart) {
    for (int i = tid; i < BM; i += NT) {
      const int64_t row = m0 + i;
      if (row < M) {
        float q = qs[0][i];
#pragma unroll
        for (int w2 = 1; w2 < WGN; ++w2) q += qs[w2][i];
        const int64_t qr = g.gcnt ? (int64_t)ymp[row] : row;  // (grouped: the Y row)
        g.qpart[(qr * g.K + k) * g.ntn + nt] = q;
      }
    }
  }
}

template <int NPROD, int KIND, int BM, int BN, int BK, int WGM = 2, int WGN = 2, int NS = 1>
__global__ __launch_bounds__(64 * WGM * WGN,
                             (Bf16Occ<BM, BN, BK, KIND, NPROD, 64 * WGM * WGN, NS>::value))
void quad_gemm_bf16_kernel(Bf16Params g) {
  bf16_tile<NPROD, KIND, BM, BN, BK, WGM, WGN, NS>(g, blockIdx.x, threadIdx.x);
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

// hi/lo split of U_k = L_k^T for K lower-triangular factors L [K][d][d]
// (row-major): U[k][n][j] = L[k][j][n] for j >= n, else 0.
__global__ void split_upper_kernel(int K, int d, const double *L, bf16_t *hi, bf16_t *lo) {
  const int64_t n_all = (int64_t)K * d * d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_all;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = i / ((int64_t)d * d);
    const int r = (int)((i / d) % d), c = (int)(i % d);  // U row r, column c
    const double v = c >= r ? L[(k * d + c) * d + r] : 0.0;
    const bf16_t h = f32_to_bf16((float)v);
    hi[i] = h;
    lo[i] = f32_to_bf16((float)(v - (double)bf16_to_f32(h)));
  }
}

}  // namespace

int launch_split_upper(int K, int d, const double *L, bf16_t *hi, bf16_t *lo, hipStream_t s) {
  const int64_t n = (int64_t)K * d * d;
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(split_upper_kernel, dim3((unsigned)std::min<int64_t>(8192, ceil_div(n, 256))),
                     dim3(256), 0, s, K, d, L, hi, lo);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

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
  // 16-byte vector access to the point rows, mu and Y
  const bool al16 = ((uintptr_t)(a.kind == 0 ? a.X : a.P0) % 16 == 0) &&
                    (a.kind == 0 || (uintptr_t)a.P1 % 16 == 0) && (uintptr_t)m.mu32 % 16 == 0 &&
                    (uintptr_t)o.Y % 16 == 0 && (a.kind == 1 || a.ldx % 4 == 0) && o.ldy % 4 == 0;
  if (!al16) {
    set_error("BF16 contraction needs 16-byte aligned X, mu and Y and row strides a multiple of 4");
    return SB_E_INVAL;
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
  p.sumsq = o.sumsq ? 1 : 0;
  p.ymap = o.ymap;
  p.ycol = o.ycol;
  p.gcnt = o.gcnt;
  p.gcap = o.gcap;
  p.yneg = o.yneg ? 1 : 0;
  p.gdst = o.gdst;
  p.gdir = (float *)o.gdir;
  p.ldg = o.ldg;
  if (o.gdst && (!o.gcnt || !o.Y || !o.gdir || o.yneg || (uintptr_t)o.gdir % 16 != 0 ||
                 o.ldg % 4 != 0 || o.ldg < m.d)) {
    set_error("direct gradient rows need grouped Y rows and a 16-byte aligned gradient");
    return SB_E_INVAL;
  }
  if (o.gcnt && (a.kind != 0 || !a.rowmap || !o.ymap || o.gcap < M)) {
    set_error("grouped contraction needs row lists of X and Y rows with capacity >= M");
    return SB_E_INVAL;
  }
  if (o.sumsq && (a.kind != 0 || !o.qpart)) {
    set_error("sum-of-squares contraction needs rows of X and a qpart output");
    return SB_E_INVAL;
  }
  o.ntn = p.ntn;
  // (grouped: each component lists at most M rows, so at most K ceil(M / BM)
  // row tiles in all; the tiles past the lists' own end return at once)
  int64_t ntile = ceil_div(M, BM) * (int64_t)(m.K * p.ntn);
  if (ntile == 0) return SB_OK;
  if (o.gcnt) ntile = ceil_div(ntile, 8) * 8;  // the grouped tile order's XCD split
  if (ntile > 0x7fffffffll) {
    set_error("contraction too large for one launch (%lld tiles)", (long long)ntile);
    return SB_E_UNSUPPORTED;
  }
  dim3 grid((unsigned)ntile);
#define SB_BF(NP, KD, BMv, BNv, BKv) \
  hipLaunchKernelGGL((quad_gemm_bf16_kernel<NP, KD, BMv, BNv, BKv>), grid, dim3(256), 0, s, p)
#define SB_BF8(NP, KD) \
  hipLaunchKernelGGL((quad_gemm_bf16_kernel<NP, KD, 256, 256, 32, 2, 4>), grid, dim3(512), 0, s, p)
#define SB_BFP(NP, BMv, BNv, WGNv) \
  hipLaunchKernelGGL((quad_gemm_bf16_kernel<NP, 0, BMv, BNv, 32, 2, WGNv, 2>), grid, \
                     dim3(128 * WGNv), 0, s, p)
#define SB_BFP1(BMv, BNv, WGNv) \
  hipLaunchKernelGGL((quad_gemm_bf16_kernel<1, 1, BMv, BNv, 32, 2, WGNv, 2>), grid, \
                     dim3(128 * WGNv), 0, s, p)
  // two LDS stages: square 32-wide tiles; for ray points the BF16 operand only
  const bool pp = t.stages == 2 && BK == 32 && BM == BN && (a.kind == 0 || nprod == 1);
  if (pp && a.kind == 1) {
    if (BM == 256) SB_BFP1(256, 256, 4);
    else SB_BFP1(128, 128, 2);
  } else if (pp && BM == 256) {
    if (nprod == 3) SB_BFP(3, 256, 256, 4);
    else SB_BFP(1, 256, 256, 4);
  } else if (pp) {
    if (nprod == 3) SB_BFP(3, 128, 128, 2);
    else SB_BFP(1, 128, 128, 2);
  } else if (a.kind == 1 && BM == 256 && BN == 256) {
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
#undef SB_BFP1
#undef SB_BFP
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
