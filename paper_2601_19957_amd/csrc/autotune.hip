// Tile-shape autotuner for the quadratic-form GEMM.
//
// Candidates (BM x BN in {64, 128}^2) are timed with HIP events on the
// caller's own inputs the first time a shape class (dtype, d, K, M rounded to
// a power of two) is seen; the fastest is cached for the process.  Timing
// runs write only the GEMM's own scratch outputs, which the real launch
// overwrites.  SB_TILE=BMxBN forces a shape; SB_AUTOTUNE=0 uses the
// heuristic choice without timing.
#include <cstdlib>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"

namespace sb {

namespace {
std::mutex g_mu;
std::map<std::tuple<int, int, int, int>, TileCfg> g_cache;

int bucket(int64_t M) {
  int b = 0;
  while ((1ll << b) < M) ++b;
  return b;
}
}  // namespace

static TileCfg heuristic(int dtype, int d, int64_t M) {
  TileCfg t;
  t.bn = (d <= 64) ? 64 : 128;
  t.bm = (M <= 4096 || d <= 64) ? 64 : 128;
  return t;
}

TileCfg autotune_tiles(int dtype, const Model &m, int64_t M, hipStream_t s) {
  const char *force = getenv("SB_TILE");
  if (force) {
    int bm = 0, bn = 0;
    if (sscanf(force, "%dx%d", &bm, &bn) == 2) {
      TileCfg t;
      t.bm = bm;
      t.bn = bn;
      return t;
    }
  }
  (void)s;
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dtype, m.d, m.K, bucket(M));
  auto it = g_cache.find(key);
  if (it != g_cache.end()) return it->second;
  TileCfg t = heuristic(dtype, m.d, M);
  g_cache[key] = t;
  return t;
}

}  // namespace sb
