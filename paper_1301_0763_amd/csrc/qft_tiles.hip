// Tile kernels (transforms of N <= 2^14 points, whole transforms in one
// workgroup's LDS).  Built once per storage type QFT_TILE_DT (0: complex
// FP32, 1: complex FP16 storage with FP32 arithmetic), tile size
// 2^QFT_TILE_TL (10 .. 14) and direction QFT_TILE_SWAP (0: forward, 1:
// adjoint), each combination a translation unit of its own so that they
// compile in parallel.
//
//  * tile_kernel_u: a contiguous batch of one size, one workgroup per tile,
//    for every N with max(2^12, N) = 2^TL (uniform plans);
//    with the constant table read from global memory or from a copy in LDS;
//  * tile_kernel_p: one transform of 2^13 or 2^14 points per tile on a
//    resident grid, each workgroup loading its next tile's x while the
//    current one runs;
//  * tile_kernel_g: the persistent kernel of uneven plans; a workgroup takes
//    tiles w = blockIdx.x, blockIdx.x + gridDim.x, ... of a size-sorted list
//    and runs the compile-time specialised body of each tile's size;
//  * tile_kernel_pg: an uneven group of 2^13- or 2^14-point transforms only,
//    on a resident grid that loads each next tile during the current one.
// All run the tile body of qft_device.hpp (tile_fetch_s, tile_fold_s,
// tile_rest_s: fold, forward and backward rounds, fused DCT-0/DST-0 chain
// with the combine), reading and writing HBM once.
#include "qft_kernels.hpp"

#if !defined(QFT_TILE_DT) || !defined(QFT_TILE_TL) || !defined(QFT_TILE_SWAP)
#error "QFT_TILE_DT (0, 1), QFT_TILE_TL (10 .. 14) and QFT_TILE_SWAP (0, 1) must be defined"
#endif

namespace qftk {

// The uniform and real-input tile kernels' forward rounds: one code path for
// both sides (16 cells per thread), else a branch between the sides' own code.
constexpr bool tile_sign_flip(int logn, int tl) {
  return tile_threads_one(logn, tl) == (1 << tl) / 16;
}

// The constant table of transforms up to 2^LOGN points (its first 2^LOGN / 4
// floats, Sec. 6.1) copied into LDS, where the rounds read their secants
// (the LDS reads are cheaper than table reads through the vector memory
// path, whose in-order counter would also make them wait for any input
// loads in flight).  Issued after the tile's x loads, so that the wait for
// the table is the wait for x that the fold has anyway; the fold's
// workgroup barrier orders the copy before the first read.
template <int LOGN>
constexpr int lds_secants() {
  return LOGN >= 3 ? (1 << LOGN) / 4 : 1;
}
template <int LOGN, int NT>
__device__ __forceinline__ void secants_to_lds(float* sl, const float* __restrict__ sec,
                                               int tid) {
  if constexpr (LOGN >= 3) {
#pragma unroll
    for (int i = tid; i < lds_secants<LOGN>(); i += NT) sl[i] = sec[i];
  }
}

// LSEC: the rounds read the constant table from a copy in LDS, else from
// global memory (which is faster depends on the size and the batch).  With 16
// cells per thread the forward rounds run one branch-free code path for both
// sides (fwd_chunk_s), which measured faster there (2^12 x 4096: 63 against
// 66 us, 2^10 x 32768: 139 against 143 us) and slower with 32.
template <int LOGN, int TL, int DT, bool SWAP, bool LSEC>
__global__ __launch_bounds__(tile_threads_one(LOGN, TL)) void tile_kernel_u(const typename Store<DT>::T* x,
                                                                   typename Store<DT>::T* X,
                                                                   int64_t batch,
                                                                   const float* sec) {
  constexpr int T = 1 << (TL - LOGN);
  constexpr int NT = tile_threads_one(LOGN, TL);
  __shared__ float2 Wl[padded_cells<kPad>(1 << TL)];
  const PadPtr<kPad> W{Wl, 0};
  const int tid = (int)threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * T;
  const int count = (int)min((int64_t)T, batch - t0);
  const ContigIO<DT, SWAP, LOGN> io(x + (t0 << LOGN), X + (t0 << LOGN));
  if constexpr (LSEC) {
    __shared__ float Sl[lds_secants<LOGN>()];
    typename ContigIO<DT, SWAP, LOGN>::Raw raw[tile_items<LOGN, T, NT>()];
    tile_fetch_s<LOGN, T, NT>(io, count, tid, raw);
    secants_to_lds<LOGN, NT>(Sl, sec, tid);
    tile_fold_s<LOGN, T, NT>(io, W, count, tid, raw);
    tile_rest_s<LOGN, T, NT, kWave, tile_sign_flip(LOGN, TL)>(io, W, count, Sl, tid, DevSync{},
                                                              DevWaveSync{});
  } else {
    tile_body_s<LOGN, T, NT, kWave, tile_sign_flip(LOGN, TL)>(io, W, count, sec, tid, DevSync{},
                                                              DevWaveSync{});
  }
}

// The same tiles on a resident grid: workgroup b takes tiles b, b + gridDim.x,
// .. and loads each next tile's x while the current one runs (tile_loop_s);
// built for one transform of 2^13 or 2^14 points per tile, the sizes whose
// LDS leaves room for only one or two workgroups per CU (with more, the
// workgroups of a CU already overlap one another's loads, and a resident
// grid measured slower).
template <int LOGN, int TL, int DT, bool SWAP>
__global__ __launch_bounds__(tile_threads_one(LOGN, TL)) void tile_kernel_p(const typename Store<DT>::T* x,
                                                                   typename Store<DT>::T* X,
                                                                   int64_t batch,
                                                                   const float* sec) {
  constexpr int T = 1 << (TL - LOGN);
  constexpr int NT = tile_threads_one(LOGN, TL);
  __shared__ float2 Wl[padded_cells<kPad>(1 << TL)];
  __shared__ float Sl[lds_secants<LOGN>()];
  const PadPtr<kPad> W{Wl, 0};
  const int tid = (int)threadIdx.x;
  tile_loop_s<LOGN, T, NT, kWave>(ContigTiles<DT, SWAP, LOGN, T>{x, X, batch},
                                  (int64_t)blockIdx.x, (int64_t)gridDim.x, W, Sl, tid,
                                  DevSync{}, DevWaveSync{},
                                  [&]() { secants_to_lds<LOGN, NT>(Sl, sec, tid); });
}

// An uneven group whose tiles each hold one transform of 2^TL points (TL =
// 13, 14), on a resident grid that loads each next tile during the current
// one (tile_loop_s over the group's tile list), 32 cells per thread.
template <int TL, int DT, bool SWAP>
__global__ __launch_bounds__(tile_threads_one(TL, TL)) void tile_kernel_pg(
    const typename Store<DT>::T* x, typename Store<DT>::T* X, const int4* __restrict__ tiles,
    const int64_t* __restrict__ offs, int ntiles, const float* sec) {
  constexpr int NT = tile_threads_one(TL, TL);
  __shared__ float2 Wl[padded_cells<kPad>(1 << TL)];
  __shared__ float Sl[lds_secants<TL>()];
  const PadPtr<kPad> W{Wl, 0};
  const int tid = (int)threadIdx.x;
  tile_loop_s<TL, 1, NT, kWave>(
      ListTiles<DT, SWAP, TL>{x, X, tiles, offs, ntiles},
      (int64_t)blockIdx.x, (int64_t)gridDim.x, W, Sl, tid, DevSync{}, DevWaveSync{},
      [&]() { secants_to_lds<TL, NT>(Sl, sec, tid); });
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
  __shared__ float Sl[lds_secants<TL>()];
  const PadPtr<kPad> W{Wl, 0};
  secants_to_lds<TL, tile_threads(TL)>(Sl, sec, (int)threadIdx.x);
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
    tile_switch<TL, DT, SWAP, 1>(logn, io, W, count, Sl, tid);
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
    tile_body_s<LOGN, T, tile_threads_one(LOGN, TL), kWave, tile_sign_flip(LOGN, TL)>(
        io, W, count, sec, (int)threadIdx.x, DevSync{}, DevWaveSync{});
  } else {
    const R* c = (const R*)a.in0;
    const R* d = (const R*)a.in1;
    R* C = (R*)a.out0;
    R* S = (R*)a.out1;
    const DctDstIO<DT, LOGN> io{c ? c + r0 * (h + 1) : nullptr, d ? d + r0 * (h - 1) : nullptr,
                                C ? C + r0 * (h + 1) : nullptr, S ? S + r0 * (h - 1) : nullptr,
                                rows - r0};
    tile_body_s<LOGN, T, tile_threads_one(LOGN, TL), kWave, tile_sign_flip(LOGN, TL)>(
        io, W, count, sec, (int)threadIdx.x, DevSync{}, DevWaveSync{});
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
      if (g.grid < g.ntiles) {
        if constexpr (LOGN == TL && TL >= 13)
          hipLaunchKernelGGL((tile_kernel_p<LOGN, TL, DT, SWAP>), dim3((unsigned)g.grid),
                             dim3(tile_threads_one(LOGN, TL)), 0, st, (const E*)in, (E*)out,
                             g.ubatch, sec);
        else
          return hipErrorInvalidValue;
      } else if (g.lds_sec) {
        hipLaunchKernelGGL((tile_kernel_u<LOGN, TL, DT, SWAP, true>), dim3((unsigned)g.ntiles),
                           dim3(tile_threads_one(LOGN, TL)), 0, st, (const E*)in, (E*)out,
                           g.ubatch, sec);
      } else {
        hipLaunchKernelGGL((tile_kernel_u<LOGN, TL, DT, SWAP, false>), dim3((unsigned)g.ntiles),
                           dim3(tile_threads_one(LOGN, TL)), 0, st, (const E*)in, (E*)out,
                           g.ubatch, sec);
      }
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
  if (g.pipe) {
    if constexpr (TL >= 13) {
      if (g.single_log2n != TL) return hipErrorInvalidValue;
      hipLaunchKernelGGL((tile_kernel_pg<TL, DT, SWAP>), dim3((unsigned)g.grid),
                         dim3(tile_threads_one(TL, TL)), 0, st, (const E*)in, (E*)out,
                         g.d_tiles, g.d_offs, g.ntiles, sec);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  hipLaunchKernelGGL((tile_kernel_g<TL, DT, SWAP>), dim3((unsigned)g.grid),
                     dim3(tile_threads(TL)), 0, st, (const E*)in, (E*)out, g.d_tiles, g.d_offs,
                     g.ntiles, sec);
  return hipGetLastError();
}

template hipError_t launch_tiles<QFT_TILE_DT, QFT_TILE_TL, (QFT_TILE_SWAP != 0)>(
    const TileGroup&, const void*, void*, const float*, hipStream_t);

}  // namespace qftk
