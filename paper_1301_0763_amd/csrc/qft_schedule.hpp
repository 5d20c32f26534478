// Host-side schedules of the improved-QFT library, shared by the GPU launcher
// (qft_lib.hip) and the CPU emulation used by the tests, so both run the very
// same sequence of passes.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace qftk {

// Constant table for transforms up to N = 2^log2n_max (N/4 entries, Sec. 6.1):
// entry L + m (L = 1, 2, 4, .., N/8; m < L) = 1/(2 cos(pi (2m+1)/(4L))), the
// secant 1/(2 cos(theta n)) of eq. qft_38A for the periodization 8L and odd
// n = 2m+1.  Evaluated in FP64 through the complement angle,
// 1/(2 sin(pi (2L-2m-1)/(4L))), so the argument never approaches the zero of
// the cosine, and rounded once to FP32.  out[0] is unused (0).
inline void fill_secants(float* out, int log2n_max) {
  const int64_t nt = ((int64_t)1 << log2n_max) / 4;
  out[0] = 0.0f;
  for (int64_t L = 1; 2 * L <= nt; L *= 2) {
    for (int64_t m = 0; m < L; ++m) {
      const double a = M_PI * (double)(2 * L - 2 * m - 1) / (double)(4 * L);
      out[L + m] = (float)(1.0 / (2.0 * std::sin(a)));
    }
  }
}

// Splits R >= 1 consecutive levels into ceil(R / kmax) chunks whose sizes
// differ by at most one (larger chunks first); returns the chunk count.
inline int level_chunks(int R, int kmax, int* sizes) {
  const int n = (R + kmax - 1) / kmax;
  for (int c = 0; c < n; ++c) sizes[c] = R / n + (c < R % n ? 1 : 0);
  return n;
}

// Most levels of one global pass (forward rounds, backward rounds, chain
// levels), at most 5 each.  Forward passes of 5 rounds hold 64 cells per
// thread (256 VGPRs, two waves per SIMD) and stream slower than a 4-round
// and a 3-round pass together; 5 backward rounds or chain levels per pass
// are faster than 4.
struct MpLevels {
  int fwd = 4, bwd = 5, chain = 5;
};

// Multi-pass schedule for transforms of length 2^logn that do not fit one
// workgroup, with LDS segments of 2^seg_log2 cells (logn >= seg_log2 + 3).
// `ex` provides:
//
//   fold()               x -> heap buffer (real fold, Sec. 4.2)
//   fwd(K, hi)           forward rounds S = 2^hi .. 2^(hi-K+1) of the blocks
//                        longer than one segment, in place
//   segment()            every 2^seg_log2 segment: its remaining forward
//                        rounds and its backward rounds in LDS; the core
//                        (both side heads) also runs the chain to
//                        P = 2^(seg_log2+1)
//   bwd(K, hi)           backward rounds S = 2^(hi-K+1) .. 2^hi, from the
//                        current heap buffer into the other one (the
//                        executor swaps them)
//   chain(K, p, first)   chain levels 2^p .. 2^(p+K-1): E values from the
//                        heap buffer (first pass) or the chain buffer (the
//                        other one), blocks from the heap buffer, outputs to
//                        the chain buffer
//   combine(K, p, first) the last chain levels (up to N) with the combine
//                        of Sec. 4.1, outputs to X
//
// Each pass runs at most `lv` rounds or levels in registers.
template <class Exec>
void multipass_schedule(Exec& ex, int logn, int seg_log2, MpLevels lv = MpLevels{}) {
  int sz[32];
  ex.fold();
  const int top = logn - 2, bottom = seg_log2 + 1;
  const int nf = level_chunks(top - bottom + 1, lv.fwd, sz);
  for (int c = 0, hi = top; c < nf; hi -= sz[c], ++c) ex.fwd(sz[c], hi);
  ex.segment();
  const int nb = level_chunks(top - bottom + 1, lv.bwd, sz);
  for (int c = nb - 1, lo = bottom; c >= 0; lo += sz[c], --c) ex.bwd(sz[c], lo + sz[c] - 1);
  const int nc = level_chunks(logn - seg_log2 - 1, lv.chain, sz);
  for (int c = 0, p = seg_log2 + 2; c < nc; p += sz[c], ++c) {
    if (c + 1 < nc) ex.chain(sz[c], p, c == 0);
    else ex.combine(sz[c], p, c == 0);
  }
}

struct TileDesc {
  int log2n;
  int first;  // index into the permuted offset list
  int count;
};

// Packed layout of an uneven batch: offsets[i] = sum of 2^log2n[j], j < i.
inline void packed_offsets(const int32_t* log2n, int64_t count, std::vector<int64_t>& offsets) {
  offsets.assign(count, 0);
  int64_t acc = 0;
  for (int64_t i = 0; i < count; ++i) {
    offsets[i] = acc;
    acc += (int64_t)1 << log2n[i];
  }
}

// Tiles of 2^tile_log2 cells for the transforms with lo <= log2n[i] <= hi
// (hi <= tile_log2), grouped by size, largest size first, each tile at most
// 2^(tile_log2 - log2n) transforms of one size; `perm` receives their element
// offsets tile by tile.  Appends to tiles/perm.
inline void build_tiles(const int32_t* log2n, const std::vector<int64_t>& offsets, int lo,
                        int hi, int tile_log2, std::vector<TileDesc>& tiles,
                        std::vector<int64_t>& perm) {
  std::vector<std::vector<int64_t>> cls(hi + 1);
  for (size_t i = 0; i < offsets.size(); ++i)
    if (log2n[i] >= lo && log2n[i] <= hi) cls[log2n[i]].push_back(offsets[i]);
  for (int lg = hi; lg >= lo; --lg) {
    const size_t per_tile = (size_t)1 << (tile_log2 - lg);
    for (size_t a = 0; a < cls[lg].size(); a += per_tile) {
      const int cnt = (int)std::min(per_tile, cls[lg].size() - a);
      tiles.push_back({lg, (int)perm.size(), cnt});
      for (int q = 0; q < cnt; ++q) perm.push_back(cls[lg][a + q]);
    }
  }
}

// Work list of an uneven plan with one tile size: transforms with
// log2n <= tile_log2 go to tiles (build_tiles), longer ones to `large`
// (index, largest first).
inline void build_uneven_worklist(const int32_t* log2n, int64_t count, int tile_log2,
                                  std::vector<int64_t>& offsets, std::vector<TileDesc>& tiles,
                                  std::vector<int64_t>& perm, std::vector<int64_t>& large) {
  packed_offsets(log2n, count, offsets);
  tiles.clear();
  perm.clear();
  large.clear();
  build_tiles(log2n, offsets, 1, tile_log2, tile_log2, tiles, perm);
  for (int64_t i = 0; i < count; ++i)
    if (log2n[i] > tile_log2) large.push_back(i);
  std::stable_sort(large.begin(), large.end(),
                   [&](int64_t a, int64_t b) { return log2n[a] > log2n[b]; });
}

}  // namespace qftk
