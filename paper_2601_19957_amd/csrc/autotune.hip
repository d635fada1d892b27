// Tile-shape autotuner for the quadratic-form GEMM.
//
// The first time a shape class (dtype, d, K, M rounded up to a power of two)
// is seen, each candidate tile (BM x BN in {64, 128}^2, the FP64 ones but
// 128 x 128 with a 32-wide k-tile, and for FP64 32 x 64 x 32; for the BF16 and
// split contractions BM x BN x k-tile in {128x128x32, 128x128x64, 256x128x32,
// 128x256x32, 256x256x32 on eight waves}, the square 32-wide ones also with
// two ping-pong LDS stages) is timed with HIP events, one warm-up and five timed launches,
// and the fastest is cached for the process.  The launches run on the
// caller's probe (its operands and scratch outputs, which the real launch
// overwrites) or, for host-level callers, on private seeded buffers of the
// shape (up to 8192 rows, values in [-1, 1)).  Timing synchronises the
// stream, so a stream under graph capture gets the heuristic choice (not
// cached).  kt = 16 restricts the FP64 and FP32 candidates to 16-wide
// k-tiles.  SB_TILE=BMxBN[xBK[xSTAGES]] forces a shape;
// SB_AUTOTUNE=0 uses the heuristic without timing.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"

namespace sb {

namespace {
std::mutex g_mu;
std::map<std::tuple<int, int, int, int, int, int>, TileCfg> g_cache;

int bucket(int64_t M) {
  int b = 0;
  while ((1ll << b) < M) ++b;
  return b;
}

// Seeded values in [-1, 1) (a 32-bit integer hash of the index).
template <typename T>
__global__ void tune_fill_kernel(int64_t n, T *p, uint32_t salt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ salt;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    const float v = (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;
    if constexpr (sizeof(T) == 2)
      p[i] = f32_to_bf16(v);
    else
      p[i] = (T)v;
  }
}

template <typename T>
void fill(int64_t n, void *p, uint32_t salt, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<int64_t>(4096, ceil_div(n, 256));
  if (n > 0) hipLaunchKernelGGL(tune_fill_kernel<T>, dim3(blocks), dim3(256), 0, s, n, (T *)p, salt);
}

TileCfg heuristic(int d, int64_t M) {
  TileCfg t;  // (for the BF16 kernels: 128 rows, 128 -> a 32-wide k-tile)
  t.bn = (d <= 64) ? 64 : 128;
  t.bm = (M <= 4096 || d <= 64) ? 64 : 128;
  return t;
}

// Times the candidates of one launch; returns false on any runtime error (the
// caller then uses the heuristic).
bool time_launches(int dtype, const Model &m, const ASrc &a, QuadOut o, int64_t M, hipStream_t s,
                   TileCfg *best, int kt) {
  const bool bf = (dtype == DT_BF16 || dtype == DT_F32S) && quad_gemm_bf16_ok(m.d);
  hipEvent_t e0, e1;
  bool ok = hipEventCreate(&e0) == hipSuccess;
  ok = ok && hipEventCreate(&e1) == hipSuccess;
  float best_ms = 0.f;
  bool have = false;
  // GEMM tiles (BM, BN); for the BF16 kernels (BM, BN, k-tile)
  const int cands[5][2] = {{64, 64}, {128, 64}, {64, 128}, {128, 128}, {32, 64}};
  const int cands_bf[7][4] = {{128, 128, 32, 1}, {128, 128, 64, 1}, {256, 128, 32, 1},
                              {128, 256, 32, 1}, {256, 256, 32, 1}, {128, 128, 32, 2},
                              {256, 256, 32, 2}};
  const int nc = bf ? 7 : (dtype == DT_F64 && kt == 32 ? 5 : 4);  // (32 x 64: FP64 only)
  for (int c = 0; c < nc && ok; ++c) {
    TileCfg t;
    t.bm = bf ? cands_bf[c][0] : cands[c][0];
    t.bn = bf ? cands_bf[c][1] : cands[c][1];
    t.bk = bf ? cands_bf[c][2] : kt;
    t.stages = bf ? cands_bf[c][3] : 1;
    // ray points run only the 32-wide k-tiles, no 256 x 128, and two stages only for
    // the BF16 operand
    if (bf && a.kind == 1 &&
        (t.bk != 32 || (t.stages != 1 && dtype != DT_BF16) || (t.bm == 256 && t.bn == 128)))
      continue;
    ok = launch_quad_gemm(dtype, m, a, M, nullptr, o, t, s) == SB_OK;  // warm-up
    ok = ok && hipEventRecord(e0, s) == hipSuccess;
    for (int r = 0; r < 5 && ok; ++r) ok = launch_quad_gemm(dtype, m, a, M, nullptr, o, t, s) == SB_OK;
    ok = ok && hipEventRecord(e1, s) == hipSuccess;
    ok = ok && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok && (!have || ms < best_ms)) {
      have = true;
      best_ms = ms;
      *best = t;
    }
  }
  if (ok) ok = hipStreamSynchronize(s) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  return ok;
}

// Times the candidates on private buffers of shape (min(M, 8192), d, K).
bool time_candidates(int dtype, int d, int K, int64_t M, hipStream_t s, TileCfg *best, int kt) {
  const int64_t Mt = std::max<int64_t>(1, std::min<int64_t>(M, 8192));
  const bool bf = (dtype == DT_BF16 || dtype == DT_F32S) && quad_gemm_bf16_ok(d);
  const size_t in_es = (dtype == DT_F64) ? 8 : 4;
  // the BF16 kernels read hi and lo copies (2 x bf16 per entry)
  const size_t op_es = (dtype == DT_F64) ? 8 : (dtype == DT_F32 ? 4 : (bf ? 4 : 2));
  const size_t acc_es = (dtype == DT_F64) ? 8 : 4;
  const size_t nX = (size_t)Mt * d, nmu = (size_t)K * d, nP = (size_t)K * d * d;
  const size_t nY = (size_t)Mt * K * d, nq = (size_t)Mt * K * ceil_div(d, 64);
  const size_t bytes = align_up(in_es * nX) + align_up(in_es * nmu) + align_up(op_es * nP) +
                       align_up(acc_es * nY) + align_up(acc_es * nq);
  void *buf = nullptr;
  if (hipMalloc(&buf, bytes) != hipSuccess) return false;
  char *p = (char *)buf;
  void *X = p;
  p += align_up(in_es * nX);
  void *mu = p;
  p += align_up(in_es * nmu);
  void *P = p;
  p += align_up(op_es * nP);
  void *Y = p;
  p += align_up(acc_es * nY);
  void *q = p;
  if (dtype == DT_F64) {
    fill<double>(nX, X, 1u, s);
    fill<double>(nmu, mu, 2u, s);
    fill<double>(nP, P, 3u, s);
  } else {
    fill<float>(nX, X, 1u, s);
    fill<float>(nmu, mu, 2u, s);
    if (dtype == DT_F32)
      fill<float>(nP, P, 3u, s);
    else
      fill<bf16_t>(bf ? 2 * nP : nP, P, 3u, s);
  }
  Model m;
  m.d = d;
  m.K = K;
  if (dtype == DT_F64) {
    m.mu64 = (const double *)mu;
    m.P64 = (const double *)P;
  } else {
    m.mu32 = (const float *)mu;
    m.Plp = P;
    if (bf) {
      m.Phi = (const bf16_t *)P;
      m.Plo = (const bf16_t *)P + nP;
    }
  }
  ASrc a;
  a.kind = 0;
  a.X = X;
  a.ldx = d;
  QuadOut o;
  o.Y = Y;
  o.ldy = (int64_t)K * d;
  o.qpart = q;
  const bool ok = time_launches(dtype, m, a, o, Mt, s, best, kt);
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  (void)hipGetLastError();
  return ok;
}
}  // namespace

bool parse_tile(const char *e, TileCfg *t) {
  int bm = 0, bn = 0, bk = 32, st = 1;
  if (!e || sscanf(e, "%dx%dx%dx%d", &bm, &bn, &bk, &st) < 2) return false;
  t->bm = bm;
  t->bn = bn;
  t->bk = bk;
  t->stages = st;
  return true;
}

TileCfg autotune_tiles(int dtype, const Model &m, int64_t M, hipStream_t s, const TuneProbe *probe,
                       bool may_alloc, int kt) {
  {
    TileCfg t;
    if (parse_tile(getenv("SB_TILE"), &t)) return t;
  }
  const char *at = getenv("SB_AUTOTUNE");
  const bool timed = !(at && at[0] == '0');
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
  auto heur = [&]() {
    TileCfg h = heuristic(m.d, M);
    if (dtype == DT_F64 || dtype == DT_F32) h.bk = kt;
    return h;
  };
  if (!timed || cs != hipStreamCaptureStatusNone || M <= 0) return heur();
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  (void)hipGetDevice(&dev);
  // (the operand kind and the sum-of-squares mode select kernels of their own)
  const int variant = (probe ? probe->a.kind + 2 * (probe->o.sumsq ? 1 : 0) : 0) + 4 * (kt != 32);
  auto key = std::make_tuple(dev, dtype, m.d, m.K, bucket(M), variant);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) return it->second;
  TileCfg t = heur();
  bool ok = false;
  if (probe)  // a prefix of the caller's launch is enough to rank the tiles
    ok = time_launches(dtype, m, probe->a, probe->o, std::min<int64_t>(M, 65536), s, &t, kt);
  else if (may_alloc)
    ok = time_candidates(dtype, m.d, m.K, M, s, &t, kt);
  else
    return t;  // no buffers to time on: heuristic, not cached
  if (!ok) t = heur();
  g_cache[key] = t;
  return t;
}

}  // namespace sb
