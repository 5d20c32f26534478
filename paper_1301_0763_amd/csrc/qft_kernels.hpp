// Definitions shared by the library's translation units: the device barrier
// functors and LDS layout constants of the kernels, and the launch interfaces
// of the persistent tile kernels (qft_tiles.hip) and of the multi-pass path
// (qft_multipass.hip), called from the plan code in qft_lib.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qft_device.hpp"
#include "qft_schedule.hpp"

namespace qftk {

struct DevSync {
  __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

// Orders the LDS accesses of one wavefront (its lanes exchange data through
// LDS between chain levels without a workgroup barrier).
struct DevWaveSync {
  __device__ __forceinline__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

constexpr int kWave = 64;
// LDS padding: one spare cell per 2^kPad = 16 cells.  Sixteen lanes reading
// consecutive cells then cover the 32 banks once; lanes owning runs of 16
// cells (fused tail) start one cell apart, runs of 8 cells (backward outputs)
// alternate between the two halves of the banks.
constexpr int kPad = 4;

// Tile kernels with tiles of 2^tl cells (10 <= tl <= 14): 16 cells per
// thread (64 to 1024 threads; 32 per thread for one transform of 2^13 or 2^14
// points, tile_threads_one), and as many resident workgroups per CU as the
// LDS (2^tl padded float2 cells out of 160 KiB) and the four waves per SIMD
// of the persistent kernel allow.
constexpr int kMinTileLog2 = 10;
constexpr int kMaxTileLog2 = 14;
constexpr int tile_threads(int tl) { return (1 << tl) / 16; }
// A tile that holds one transform of 2^13 or 2^14 points runs 32 cells per
// thread: four rounds per LDS pass instead of three (sweep_kc), which saves
// two of its seven round passes.  At 2^12 it would save none and halve the
// waves.
constexpr int tile_threads_one(int logn, int tl) {
  return (logn == tl && tl >= 13) ? (1 << tl) / 32 : (1 << tl) / 16;
}
constexpr int tile_wgs_per_cu(int tl) {
  return tl <= 10 ? 16 : (tl == 11 ? 8 : (tl == 12 ? 4 : (tl == 13 ? 2 : 1)));
}

// One tile-kernel launch.  Uniform groups (d_tiles == nullptr): a
// contiguous batch of `ubatch` transforms of 2^ulog2n points in tiles of
// T = 2^(tl - ulog2n) transforms (the last one ragged), one workgroup per
// tile (grid = ntiles) or, for one transform of 2^13 or 2^14 points per
// tile, `grid` < ntiles resident workgroups striding over them and loading
// each next tile during the current one (tl = max(10, ulog2n)); lds_sec:
// the rounds read the constant table from a copy in LDS (always so on a
// resident grid).  Uneven groups: tile w = (log2n, first,
// count, 0) holds `count` transforms of 2^log2n points at element offsets
// d_offs[first .. first + count); `grid` workgroups stride over the tiles
// (grid = ntiles: one workgroup per tile) and exit after their last one.
struct TileGroup {
  int tl;
  int ntiles;
  int grid;
  int4* d_tiles;
  int64_t* d_offs;
  int ulog2n;
  int64_t ubatch;
  int64_t rows;  // real-input plans: real signals (2 per transform slot)
  bool lds_sec = false;
  // uneven groups: the one size of all its tiles (0 if several), and whether
  // such a group of 2^13- or 2^14-point transforms runs on a resident grid
  // that loads each next tile during the current one
  int single_log2n = 0;
  bool pipe = false;
};

// Pointers of a real-input exec: rdft in0 -> out0; DCT-0/DST-0 in0 (c) ->
// out0 (C) and in1 (d) -> out1 (S), either pair may be null.
struct RealArgs {
  const void* in0;
  const void* in1;
  void* out0;
  void* out1;
};

// Launches one group with the tile kernels of storage type DT (0: complex
// FP32, 1: complex FP16), tile size 2^TL and direction SWAP (adjoint).
// Defined in qft_tiles.hip and explicitly instantiated there once per
// (DT, TL, SWAP), each in a translation unit of its own.
template <int DT, int TL, bool SWAP>
hipError_t launch_tiles(const TileGroup& g, const void* in, void* out, const float* sec,
                        hipStream_t st);

// Launches a uniform group of a real-input plan: kind 0 = rdft, 1 = DCT-0 /
// DST-0 (qft_tiles.hip, instantiated in the forward translation units).
template <int DT, int TL>
hipError_t launch_real(const TileGroup& g, int kind, const RealArgs& a, const float* sec,
                       hipStream_t st);

// Multi-pass path (qft_multipass.hip, one translation unit per storage type
// DT): `batch` contiguous transforms of 2^log2n points, kMpSegLog2 + 3 <=
// log2n <= 24 (swap: the adjoint), or `rows` real signals of a real-input
// plan (kind as in launch_real; two signals per transform slot).  W0 and
// W1 are heap buffers of (transforms or slots) * 2^log2n cells each.  `seg`:
// log2 of the LDS segment, 12 or 13 (log2n >= seg + 3); real-input plans use
// kMpSegLog2.
constexpr int kMpSegLog2 = 12;  // default LDS segment of the multi-pass path

template <int DT>
hipError_t launch_multipass(bool swap, const void* in, void* out, int log2n, int64_t batch,
                            const float* sec, float2* W0, float2* W1, MpLevels lv, int seg,
                            hipStream_t st);

template <int DT>
hipError_t launch_multipass_real(int kind, const RealArgs& a, int log2n, int64_t rows,
                                 const float* sec, float2* W0, float2* W1, hipStream_t st);

// Fixed-point (QFT_I32) transforms of 2^log2n points (1 <= log2n <=
// kFixedMaxLog2), `batch` of them, complex int32 pairs in and out; H and
// shift are the device copies of fx::fill_table_q's table; scratch holds
// 2 * batch * 2^log2n int2 cells when log2n > 12 (else unused).
constexpr int kFixedMaxLog2 = 16;
hipError_t launch_fixed(bool swap, const void* in, void* out, int log2n, int64_t batch,
                        const int* H, const int* shift, int2* scratch, hipStream_t st);

}  // namespace qftk
