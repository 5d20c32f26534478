// Tile kernels (transforms of N <= 2^14 points, whole transforms in one
// workgroup's LDS).  Built once per storage type QFT_TILE_DT (0: complex
// FP32, 1: complex FP16 storage with FP32 arithmetic), tile size
// 2^QFT_TILE_TL (12, 13, 14) and direction QFT_TILE_SWAP (0: forward, 1:
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
#error "QFT_TILE_DT (0, 1), QFT_TILE_TL (12, 13, 14) and QFT_TILE_SWAP (0, 1) must be defined"
#endif

namespace qftk {

template <int LOGN, int TL, int DT, bool SWAP>
__global__ __launch_bounds__(tile_threads(TL)) void tile_kernel_u(const typename Store<DT>::T* x,
                                                                   typename Store<DT>::T* X,
                                                                   int64_t batch,
                                                                   const float* sec) {
  constexpr int T = 1 << (TL - LOGN);
  __shared__ float2 Wl[padded_cells<kPad>(1 << TL)];
  const PadPtr<kPad> W{Wl, 0};
  const int64_t t0 = (int64_t)blockIdx.x * T;
  const int count = (int)min((int64_t)T, batch - t0);
  const ContigIO<DT, SWAP, LOGN> io(x + (t0 << LOGN), X + (t0 << LOGN));
  tile_body_s<LOGN, T, tile_threads(TL), kWave>(io, W, count, sec, (int)threadIdx.x, DevSync{},
                                                DevWaveSync{});
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
    const GatherIO<DT, SWAP> io(x, X, offs + __builtin_amdgcn_readfirstlane(d.y));
    // The thread index is laundered once per tile: otherwise the compiler
    // hoists every thread-dependent LDS address of the bodies out of the
    // loop and keeps them all live (hundreds of registers, spills).
    int tid = (int)threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
    tile_switch<TL, DT, SWAP, 1>(logn, io, W, count, sec, tid);
    __syncthreads();
  }
}

template <int DT, int TL, bool SWAP, int LOGN>
hipError_t launch_uniform(const TileGroup& g, const void* in, void* out, const float* sec,
                          hipStream_t st) {
  using E = typename Store<DT>::T;
  if constexpr (LOGN <= TL) {
    if (g.ulog2n != LOGN) return launch_uniform<DT, TL, SWAP, LOGN + 1>(g, in, out, sec, st);
    if constexpr ((LOGN < kMinTileLog2 ? kMinTileLog2 : LOGN) == TL) {
      hipLaunchKernelGGL((tile_kernel_u<LOGN, TL, DT, SWAP>), dim3((unsigned)g.ntiles),
                         dim3(tile_threads(TL)), 0, st, (const E*)in, (E*)out, g.ubatch, sec);
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
