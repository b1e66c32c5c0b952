// Solve-kernel variants and the autotuned choice per (precision, block size).
#pragma once
#include <stddef.h>

namespace fb {

// variant v: tile width (16 or 32 right-hand sides), whether the factor
// fragments of the next block product are prefetched into registers, how
// many 16-column tiles one wave computes (2 for v = 4, 5, with registers
// capped for two waves per SIMD in complex64), and for v = 6, 7 (16-column tiles)
// registers capped for three waves per SIMD; v = 8, 9 (16- and 32-column
// tiles) stream their factor fragments chunk by chunk instead
constexpr int kNumVariants = 10;
inline int variant_tile(int v) { return ((v >= 2 && v < 6) || v == 9) ? 32 : 16; }
inline bool variant_prefetch(int v) { return (v & 1) != 0; }
inline int variant_nc(int v) { return (v == 4 || v == 5) ? 2 : 1; }
inline bool variant_streamed(int v) { return v >= 8; }
// a streamed variant is chosen only when it takes under this fraction of the
// best other variant's time
constexpr float kStreamedMargin = 0.97f;
// dynamic LDS of the block-solve kernel: the block's permutation and its
// inverse (2 NB entries each) and three NB x T slots of the factors' element
// type with rows padded to T + 1
inline size_t solve_lds_bytes(int nb, int t, size_t elem) {
  return ((4 * (size_t)nb * sizeof(int) + 15) & ~(size_t)15) + (size_t)3 * nb * (t + 1) * elem;
}
bool variant_fits(size_t rsize, int nb, int v);
int tuned_variant(size_t rsize, int nb);
void set_tuned_variant(size_t rsize, int nb, int v);

}  // namespace fb
