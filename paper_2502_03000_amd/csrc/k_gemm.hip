// Plain-precision GEMM / SYRK launchers (FP32 and FP64 MFMA) and the tile
// heuristics the planner uses to size split-K workspace.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gemm_device.h"
#include "kernels.h"

namespace hexla {
namespace k {

namespace {

struct Tile {
  int bm, bn, bk;
};
// FP32: 0 = 128x128, 1 = 128x64 (skinny N), 2 = 64x64 (small), then the
// same shapes with BK = 32 (longer steps: more bytes in flight per step),
// then 64x64 with BK = 64 and 128: a split-K chunk of a long, narrow product
// arrives in one or two steps, so a workgroup waits for memory once or twice
// instead of once per short step
constexpr Tile kTilesF32[] = {{128, 128, 16}, {128, 64, 16}, {64, 64, 16}, {128, 128, 32},
                              {128, 64, 32},  {64, 64, 32},  {64, 64, 64}, {64, 64, 128}};
// FP64: 0 = 64x64x16, 1 = 128x128x8, 2 = 128x128x8 held to 256 registers per
// wave (two workgroups per CU instead of one), 3 = 128x128x16 (one wave per
// SIMD; a longer step hides more of each step's load latency)
constexpr Tile kTilesF64[] = {{64, 64, 16}, {128, 128, 8}, {128, 128, 8}, {128, 128, 16}};

typedef void (*GemmFn)(GemmArgs);

template <typename T, int BM, int BN, int BK, int WPE = 1>
GemmFn pick(bool ta, bool tb, bool vec) {
  if (vec) {
    if (ta) return tb ? gemm_kernel<T, true, true, BM, BN, BK, true, WPE> : gemm_kernel<T, true, false, BM, BN, BK, true, WPE>;
    return tb ? gemm_kernel<T, false, true, BM, BN, BK, true, WPE> : gemm_kernel<T, false, false, BM, BN, BK, true, WPE>;
  }
  if (ta) return tb ? gemm_kernel<T, true, true, BM, BN, BK, false, WPE> : gemm_kernel<T, true, false, BM, BN, BK, false, WPE>;
  return tb ? gemm_kernel<T, false, true, BM, BN, BK, false, WPE> : gemm_kernel<T, false, false, BM, BN, BK, false, WPE>;
}

GemmFn kernel_for(int dtype, int tile, bool ta, bool tb, bool vec) {
  if (dtype == 1) {
    switch (tile) {
      case 0: return pick<float, 128, 128, 16>(ta, tb, vec);
      case 1: return pick<float, 128, 64, 16>(ta, tb, vec);
      case 2: return pick<float, 64, 64, 16>(ta, tb, vec);
      case 3: return pick<float, 128, 128, 32>(ta, tb, vec);
      case 4: return pick<float, 128, 64, 32>(ta, tb, vec);
      case 5: return pick<float, 64, 64, 32>(ta, tb, vec);
      case 6: return pick<float, 64, 64, 64>(ta, tb, vec);
      default: return pick<float, 64, 64, 128>(ta, tb, vec);
    }
  }
  switch (tile) {
    case 1: return pick<double, 128, 128, 8>(ta, tb, vec);
    case 2: return pick<double, 128, 128, 8, 2>(ta, tb, vec);
    case 3: return pick<double, 128, 128, 16>(ta, tb, vec);
    default: return pick<double, 64, 64, 16>(ta, tb, vec);
  }
}

Tile tile_of(int dtype, int tile) { return dtype == 1 ? kTilesF32[tile] : kTilesF64[tile]; }

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

int gemm_tile_count(int dtype) { return dtype == 1 ? 8 : 4; }

void gemm_tile_shape(int dtype, int precision, int tile, int* bm, int* bn, int* bk) {
  if (precision != GEMM_PLAIN) {  // split-BF16 family: one 128 x 128 x 32 tile
    *bm = 128;
    *bn = 128;
    *bk = 32;
    return;
  }
  const Tile t = tile_of(dtype, tile);
  *bm = t.bm;
  *bn = t.bn;
  *bk = t.bk;
}

int64_t gemm_tiles_for(int dtype, int tile, int mode, int64_t m, int64_t n) {
  const Tile t = tile_of(dtype, tile);
  if (mode == 1) {
    const int64_t tt = cdiv(n, t.bn);
    return tt * (tt + 1) / 2;
  }
  return cdiv(m, t.bm) * cdiv(n, t.bn);
}

bool gemm_tile_valid(int dtype, int tile, int mode) {
  if (tile < 0 || tile >= gemm_tile_count(dtype)) return false;
  const Tile t = tile_of(dtype, tile);
  return mode != 1 || t.bm == t.bn;
}

// Split count giving about `target` workgroups with at least `min_steps` BK
// steps each; the chunk is a multiple of BK.
int gemm_split_for(int dtype, int tile, int mode, int64_t m, int64_t n, int64_t k,
                   int64_t target, int64_t min_steps) {
  const Tile t = tile_of(dtype, tile);
  const int64_t tiles = gemm_tiles_for(dtype, tile, mode, m, n);
  int64_t split = 1;
  if (tiles < target) split = cdiv(target, tiles);
  split = std::min<int64_t>(split, std::max<int64_t>(1, k / (min_steps * t.bk)));
  split = std::min<int64_t>(split, 64);
  if (split > 1) {
    const int64_t chunk = cdiv(cdiv(k, split), t.bk) * t.bk;
    split = cdiv(k, chunk);
  }
  return int(std::max<int64_t>(split, 1));
}

GemmConfig gemm_choose(int dtype, int precision, int mode, int64_t m, int64_t n, int64_t k) {
  GemmConfig c{0, 1};
  if (precision != GEMM_PLAIN) return gemm_choose_split(dtype, precision, mode, m, n, k);
  if (dtype == 1) {
    if (mode == 1) c.tile = (n >= 1024) ? 3 : 5;
    else if (m <= 64 || (n <= 64 && m < 1024)) c.tile = 5;
    else if (n <= 64) c.tile = 4;
    else c.tile = (m * n >= 1024 * 1024) ? 3 : 5;
  } else {
    c.tile = (m * n >= int64_t(2048) * 2048) ? 2 : 0;
  }
  c.split = gemm_split_for(dtype, c.tile, mode, m, n, k, 256, 8);
  return c;
}

size_t gemm_partial_bytes(int dtype, const GemmConfig& cfg, int64_t m, int64_t n) {
  if (cfg.split <= 1) return 0;
  const size_t esz = dtype == 0 ? 8 : 4;
  return size_t(cfg.split) * size_t(m) * size_t(n) * esz;
}

hipError_t gemm_launch(int dtype, int precision, int mode, int ta, int tb, int64_t m, int64_t n,
                       int64_t k, double alpha, const void* A, int64_t lda, const void* B,
                       int64_t ldb, double beta, void* C, int64_t ldc, void* partial,
                       const GemmConfig& cfg, hipStream_t s) {
  if (m == 0 || n == 0) return hipSuccess;
  if (precision != GEMM_PLAIN)
    return gemm_split_launch(dtype, precision, mode, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta,
                             C, ldc, partial, cfg, s);
  const Tile t = tile_of(dtype, cfg.tile);
  GemmArgs g{};
  g.m = m; g.n = n; g.k = k;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.partial = partial;
  g.mode = mode;
  g.split = cfg.split;
  g.k_chunk = cdiv(cdiv(k, cfg.split), t.bk) * t.bk;
  if (g.k_chunk == 0) g.k_chunk = t.bk;
  g.tiles_m = int(cdiv(m, t.bm));
  g.tiles_n = int(cdiv(n, t.bn));
  const int esz = dtype == 0 ? 8 : 4;
  const int vw = 16 / esz;
  const bool vec = (lda % vw == 0) && (ldb % vw == 0) &&
                   (reinterpret_cast<uintptr_t>(A) % 16 == 0) &&
                   (reinterpret_cast<uintptr_t>(B) % 16 == 0);
  int64_t blocks;
  if (mode == 1) {
    const int64_t tt = g.tiles_n;
    blocks = tt * (tt + 1) / 2;
  } else {
    blocks = int64_t(g.tiles_m) * g.tiles_n;
  }
  GemmFn fn = kernel_for(dtype, cfg.tile, ta != 0, tb != 0, vec);
  hipLaunchKernelGGL(fn, dim3(unsigned(blocks), unsigned(cfg.split)), dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || cfg.split <= 1) return e;
  return dtype == 0 ? splitk_reduce_launch<double>(g, s) : splitk_reduce_launch<float>(g, s);
}

}  // namespace k
}  // namespace hexla
