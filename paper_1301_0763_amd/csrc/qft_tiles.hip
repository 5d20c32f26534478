// Tile kernels (transforms of N <= 2^14 points, whole transforms in one
// workgroup's LDS).  Built once per storage type QFT_TILE_DT (0: complex
// FP32, 1: complex FP16 storage with FP32 arithmetic), tile size
// 2^QFT_TILE_TL (10 .. 14) and direction QFT_TILE_SWAP (0: forward, 1:
// adjoint), each combination a translation unit of its own so that they
// compile in parallel.
//
//  * tile_kernel_u: a contiguous batch of one size, one workgroup per tile,
//    for every N with max(2^12, N) = 2^TL (uniform plans);
//  * tile_kernel_g: the persistent kernel of uneven plans; a workgroup takes
//    tiles w = blockIdx.x, blockIdx.x + gridDim.x, ... of a size-sorted list
//    and runs the compile-time specialised body of each tile's size.
// Both run qftk::tile_body_s (fold, forward and backward rounds, fused
// DCT-0/DST-0 chain with the combine), reading and writing HBM once.
#include "qft_kernels.hpp"

#if !defined(QFT_TILE_DT) || !defined(QFT_TILE_TL) || !defined(QFT_TILE_SWAP)
#error "QFT_TILE_DT (0, 1), QFT_TILE_TL (10 .. 14) and QFT_TILE_SWAP (0, 1) must be defined"
#endif

namespace qftk {

template <int LOGN, int TL, int DT, bool SWAP>
__global__ __launch_bounds__(tile_threads_one(LOGN, TL)) void tile_kernel_u(const typename Store<DT>::T* x,
                                                                   typename Store<DT>::T* X,
                                                                   int64_t batch,
                                                                   const float* sec) {
  constexpr int T = 1 << (TL - LOGN);
  __shared__ float2 Wl[padded_cells<kPad>(1 << TL)];
  const PadPtr<kPad> W{Wl, 0};
  const int64_t t0 = (int64_t)blockIdx.x * T;
  const int count = (int)min((int64_t)T, batch - t0);
  const ContigIO<DT, SWAP, LOGN> io(x + (t0 << LOGN), X + (t0 << LOGN));
  tile_body_s<LOGN, T, tile_threads_one(LOGN, TL), kWave>(io, W, count, sec, (int)threadIdx.x,
                                                          DevSync{}, DevWaveSync{});
}

template <int TL, int DT, bool SWAP, int LOGN>
__device__ __forceinline__ void tile_switch(int logn, const GatherIO<DT, SWAP>& io,
                                            PadPtr<kPad> W, int count, const float* sec,
                                            int tid) {
  if constexpr (LOGN <= TL) {
    if (logn == LOGN) {
      tile_body_s<LOGN, (1 << (TL - LOGN)), tile_threads(TL), kWave>(io, W, count, sec, tid,
                                                                     DevSync{}, DevWaveSync{});
    } else {
      tile_switch<TL, DT, SWAP, LOGN + 1>(logn, io, W, count, sec, tid);
    }
  }
}

// 4 waves per SIMD: the resident workgroups that the LDS allows (4, 2, 1).
template <int TL, int DT, bool SWAP>
__global__ __launch_bounds__(tile_threads(TL), 4) void tile_kernel_g(
    const typename Store<DT>::T* x, typename Store<DT>::T* X, const int4* __restrict__ tiles,
    const int64_t* __restrict__ offs, int ntiles, const float* sec) {
  __shared__ float2 Wl[padded_cells<kPad>(1 << TL)];
  const PadPtr<kPad> W{Wl, 0};
  for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
    // the descriptor is the same for the whole workgroup: broadcast it from
    // lane 0, so that the size dispatch below is a uniform (scalar) branch
    const int4 d = tiles[w];
    const int logn = __builtin_amdgcn_readfirstlane(d.x);
    const int count = __builtin_amdgcn_readfirstlane(d.z);
    const GatherIO<DT, SWAP> io(x, X, offs + __builtin_amdgcn_readfirstlane(d.y), logn);
    // The thread index is laundered once per tile: otherwise the compiler
    // hoists every thread-dependent LDS address of the bodies out of the
    // loop and keeps them all live (hundreds of registers, spills).
    int tid = (int)threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
    tile_switch<TL, DT, SWAP, 1>(logn, io, W, count, sec, tid);
    __syncthreads();
  }
}

// Real-input kernels (KIND 0: rdft of real signals, KIND 1: DCT-0 and DST-0),
// two real signals per transform slot, one workgroup per tile of T slots.
template <int LOGN, int TL, int DT, int KIND>
__global__ __launch_bounds__(tile_threads_one(LOGN, TL)) void tile_kernel_r(RealArgs a, int64_t rows,
                                                                   int64_t slots,
                                                                   const float* sec) {
  constexpr int T = 1 << (TL - LOGN);
  constexpr int n = 1 << LOGN, h = n >> 1;
  using R = typename RStore<DT>::T;
  __shared__ float2 Wl[padded_cells<kPad>(1 << TL)];
  const PadPtr<kPad> W{Wl, 0};
  const int64_t t0 = (int64_t)blockIdx.x * T;
  const int count = (int)min((int64_t)T, slots - t0);
  const int64_t r0 = 2 * t0;  // first real signal of the tile
  if constexpr (KIND == 0) {
    using E = typename Store<DT>::T;
    const RealPairIO<DT, LOGN> io{(const R*)a.in0 + r0 * n, (E*)a.out0 + r0 * (h + 1), rows - r0};
    tile_body_s<LOGN, T, tile_threads_one(LOGN, TL), kWave>(io, W, count, sec, (int)threadIdx.x,
                                                            DevSync{}, DevWaveSync{});
  } else {
    const R* c = (const R*)a.in0;
    const R* d = (const R*)a.in1;
    R* C = (R*)a.out0;
    R* S = (R*)a.out1;
    const DctDstIO<DT, LOGN> io{c ? c + r0 * (h + 1) : nullptr, d ? d + r0 * (h - 1) : nullptr,
                                C ? C + r0 * (h + 1) : nullptr, S ? S + r0 * (h - 1) : nullptr,
                                rows - r0};
    tile_body_s<LOGN, T, tile_threads_one(LOGN, TL), kWave>(io, W, count, sec, (int)threadIdx.x,
                                                            DevSync{}, DevWaveSync{});
  }
}

template <int DT, int TL, int KIND, int LOGN>
hipError_t launch_real_n(const TileGroup& g, const RealArgs& a, const float* sec,
                         hipStream_t st) {
  if constexpr (LOGN <= TL) {
    if (g.ulog2n != LOGN) return launch_real_n<DT, TL, KIND, LOGN + 1>(g, a, sec, st);
    if constexpr ((LOGN < kMinTileLog2 ? kMinTileLog2 : LOGN) == TL) {
      hipLaunchKernelGGL((tile_kernel_r<LOGN, TL, DT, KIND>), dim3((unsigned)g.ntiles),
                         dim3(tile_threads_one(LOGN, TL)), 0, st, a, g.rows, g.ubatch, sec);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <int DT, int TL>
hipError_t launch_real(const TileGroup& g, int kind, const RealArgs& a, const float* sec,
                       hipStream_t st) {
  if (g.tl != TL || g.ntiles <= 0 || g.d_tiles) return hipErrorInvalidValue;
  return kind == 0 ? launch_real_n<DT, TL, 0, 1>(g, a, sec, st)
                   : launch_real_n<DT, TL, 1, 1>(g, a, sec, st);
}

#if QFT_TILE_SWAP == 0
template hipError_t launch_real<QFT_TILE_DT, QFT_TILE_TL>(const TileGroup&, int, const RealArgs&,
                                                          const float*, hipStream_t);
#endif

template <int DT, int TL, bool SWAP, int LOGN>
hipError_t launch_uniform(const TileGroup& g, const void* in, void* out, const float* sec,
                          hipStream_t st) {
  using E = typename Store<DT>::T;
  if constexpr (LOGN <= TL) {
    if (g.ulog2n != LOGN) return launch_uniform<DT, TL, SWAP, LOGN + 1>(g, in, out, sec, st);
    if constexpr ((LOGN < kMinTileLog2 ? kMinTileLog2 : LOGN) == TL) {
      hipLaunchKernelGGL((tile_kernel_u<LOGN, TL, DT, SWAP>), dim3((unsigned)g.ntiles),
                         dim3(tile_threads_one(LOGN, TL)), 0, st, (const E*)in, (E*)out,
                         g.ubatch, sec);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <int DT, int TL, bool SWAP>
hipError_t launch_tiles(const TileGroup& g, const void* in, void* out, const float* sec,
                        hipStream_t st) {
  using E = typename Store<DT>::T;
  if (g.tl != TL || g.ntiles <= 0) return hipErrorInvalidValue;
  if (!g.d_tiles) return launch_uniform<DT, TL, SWAP, 1>(g, in, out, sec, st);
  if (g.grid <= 0 || g.grid > g.ntiles) return hipErrorInvalidValue;
  hipLaunchKernelGGL((tile_kernel_g<TL, DT, SWAP>), dim3((unsigned)g.grid),
                     dim3(tile_threads(TL)), 0, st, (const E*)in, (E*)out, g.d_tiles, g.d_offs,
                     g.ntiles, sec);
  return hipGetLastError();
}

template hipError_t launch_tiles<QFT_TILE_DT, QFT_TILE_TL, (QFT_TILE_SWAP != 0)>(
    const TileGroup&, const void*, void*, const float*, hipStream_t);

}  // namespace qftk
