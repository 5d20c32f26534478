// Multi-pass path: transforms longer than one workgroup's LDS (the library
// runs N = 2^17 .. 2^24 complex, and real-input N = 2^15 .. 2^24, here),
// built once per storage type QFT_MP_DT (0: FP32, 1: FP16).  The passes of
// multipass_schedule (qft_schedule.hpp) over two heap buffers:
//
//   fold        x -> heap (through the plan's IO accessor)
//   fwd         up to 4 forward rounds of the large blocks per pass, in
//               registers, in place
//   segment     one workgroup per segment index (2^12 or 2^13 cells, a
//               schedule's choice): the segment of both sides, its remaining
//               forward and its backward rounds in LDS; workgroup 0 of a
//               transform takes both side heads and also runs the chain to
//               twice the segment
//   bwd         up to 5 backward rounds per pass, heap -> other buffer
//   chain       up to 5 chain levels per pass, E values and outputs in the
//               chain buffer, DCT-II / DST-II blocks read from the heap
//   combine     the last chain levels with the combine, straight into X
#include "qft_kernels.hpp"
#include "qft_schedule.hpp"

#if !defined(QFT_MP_DT)
#error "QFT_MP_DT (0, 1) must be defined"
#endif

namespace qftk {

constexpr int MP_BLOCK = 256;

#define QFT_GRID_STRIDE(i, total)                                              \
  for (int64_t i = (int64_t)blockIdx.x * MP_BLOCK + threadIdx.x; i < (total); \
       i += (int64_t)gridDim.x * MP_BLOCK)

template <class IO>
__global__ __launch_bounds__(MP_BLOCK) void mp_fold_kernel(IO io, float2* W, int logn,
                                                           int64_t batch) {
  QFT_GRID_STRIDE(i, batch << (logn - 1)) mp_fold_io_item(io, W, logn, i);
}

template <int K>
__global__ __launch_bounds__(MP_BLOCK) void mp_fwd_kernel(float2* W, int logn, int64_t batch,
                                                          int hi, const float* sec) {
  QFT_GRID_STRIDE(i, (2 * batch) << (logn - K - 2)) mp_fwd_item<K>(W, logn, hi, sec, i);
}

// Backward rounds 2^(hi-K+1) .. 2^hi, one wavefront's 64 items at a time
// (mp_bwd_wave_item); each wave stages its outputs in its own LDS rows.  The
// launch guarantees hi - K >= 6 and a multiple of MP_BLOCK items.
template <int K>
__global__ __launch_bounds__(MP_BLOCK) void mp_bwd_kernel(const float2* Win, float2* Wout,
                                                          int logn, int64_t batch, int hi) {
  constexpr int ROW = MpBwdStage<K>::ROW;
  __shared__ float2 stage[MP_BLOCK * ROW];
  const int lane = (int)threadIdx.x & (kWave - 1);
  float2* ws = stage + ((int)threadIdx.x - lane) * ROW;
  const int64_t total = (2 * batch) << (logn - 1 - K);
  for (int64_t b = (int64_t)blockIdx.x * MP_BLOCK; b < total; b += (int64_t)gridDim.x * MP_BLOCK)
    mp_bwd_wave_item<K, kWave>(Win, Wout, ws, logn, hi, b + threadIdx.x, lane, DevWaveSync{});
}

// E and Wout may be the same buffer (see mp_chain_item).
template <int K>
__global__ __launch_bounds__(MP_BLOCK) void mp_chain_kernel(const float2* E, const float2* O,
                                                            float2* Wout, int logn,
                                                            int64_t batch, int p) {
  QFT_GRID_STRIDE(i, batch << (p - 2)) mp_chain_item<K>(E, O, Wout, logn, p, i);
}

template <int K, class IO>
__global__ __launch_bounds__(MP_BLOCK) void mp_combine_kernel(IO io, const float2* E,
                                                              const float2* O, int logn,
                                                              int64_t batch, int p) {
  QFT_GRID_STRIDE(i, batch << (p - 2)) mp_chain_combine_item<K>(io, E, O, logn, p, i);
}

#undef QFT_GRID_STRIDE

// Segment pass: workgroup (t, j) takes segment j of both sides of transform
// t (j = 0: the side heads and the top cell), 32 cells per thread (four
// rounds per LDS pass).
template <int MC_LOG2, int BLOCK>
__global__ __launch_bounds__(BLOCK) void mp_segment_kernel(float2* W, int logn,
                                                           const float* sec) {
  constexpr int MC = 1 << MC_LOG2;
  static_assert(2 * MC == 32 * BLOCK, "32 cells per thread");
  __shared__ float2 Ll[padded_cells<kPad>(2 * MC + 1)];
  const PadPtr<kPad> L{Ll, 0};
  const int lgsegs = logn - 1 - MC_LOG2;
  const int64_t t = (int64_t)blockIdx.x >> lgsegs;
  const int j = (int)(blockIdx.x & ((1u << lgsegs) - 1));
  mp_segment_pair<MC_LOG2, BLOCK, kWave>(W + (t << logn), L, 1 << (logn - 1), j, sec,
                                         (int)threadIdx.x, DevSync{}, DevWaveSync{});
}

namespace {

unsigned grid_for(int64_t work) {
  int64_t g = (work + MP_BLOCK - 1) / MP_BLOCK;
  const int64_t cap = 1 << 20;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// GPU executor of multipass_schedule (passes of 1 to kMpMaxLevels rounds or
// chain levels).
template <class IO>
struct GpuMultipass {
  IO io;
  int logn;
  int64_t batch;
  const float* sec;
  float2* cur;  // heap buffer
  float2* oth;  // the other buffer (backward output, then chain buffer)
  int seg;      // log2 of the LDS segment (12 or 13)
  hipStream_t st;
  hipError_t err = hipSuccess;

  void fold() {
    hipLaunchKernelGGL((mp_fold_kernel<IO>), dim3(grid_for(batch << (logn - 1))),
                       dim3(MP_BLOCK), 0, st, io, cur, logn, batch);
  }
  template <int K>
  void fwd_k(int hi) {
    hipLaunchKernelGGL((mp_fwd_kernel<K>), dim3(grid_for((2 * batch) << (logn - K - 2))),
                       dim3(MP_BLOCK), 0, st, cur, logn, batch, hi, sec);
  }
  void fwd(int K, int hi) {
    switch (K) {
      case 1: fwd_k<1>(hi); break;
      case 2: fwd_k<2>(hi); break;
      case 3: fwd_k<3>(hi); break;
      case 4: fwd_k<4>(hi); break;
      case 5: fwd_k<5>(hi); break;
      default: err = hipErrorInvalidValue; break;
    }
  }
  void segment() {
    const int64_t blocks = batch << (logn - 1 - seg);
    if (seg == 13)
      hipLaunchKernelGGL((mp_segment_kernel<13, 512>), dim3((unsigned)blocks), dim3(512), 0, st,
                         cur, logn, sec);
    else
      hipLaunchKernelGGL((mp_segment_kernel<12, 256>), dim3((unsigned)blocks), dim3(256), 0, st,
                         cur, logn, sec);
  }
  template <int K>
  void bwd_k(int hi) {
    // the kernel's wave staging: a segment (2^(hi-K) items) holds whole
    // wavefronts, and the items fill whole workgroups
    if (hi - K < 6 || logn - 1 - K < 8) {
      err = hipErrorInvalidValue;
      return;
    }
    hipLaunchKernelGGL((mp_bwd_kernel<K>), dim3(grid_for((2 * batch) << (logn - 1 - K))),
                       dim3(MP_BLOCK), 0, st, (const float2*)cur, oth, logn, batch, hi);
    std::swap(cur, oth);
  }
  void bwd(int K, int hi) {
    switch (K) {
      case 1: bwd_k<1>(hi); break;
      case 2: bwd_k<2>(hi); break;
      case 3: bwd_k<3>(hi); break;
      case 4: bwd_k<4>(hi); break;
      case 5: bwd_k<5>(hi); break;
      default: err = hipErrorInvalidValue; break;
    }
  }
  template <int K>
  void chain_k(int p, bool first) {
    hipLaunchKernelGGL((mp_chain_kernel<K>), dim3(grid_for(batch << (p - 2))), dim3(MP_BLOCK), 0,
                       st, (const float2*)(first ? cur : oth), (const float2*)cur, oth, logn,
                       batch, p);
  }
  void chain(int K, int p, bool first) {
    switch (K) {
      case 1: chain_k<1>(p, first); break;
      case 2: chain_k<2>(p, first); break;
      case 3: chain_k<3>(p, first); break;
      case 4: chain_k<4>(p, first); break;
      case 5: chain_k<5>(p, first); break;
      default: err = hipErrorInvalidValue; break;
    }
  }
  template <int K>
  void combine_k(int p, bool first) {
    hipLaunchKernelGGL((mp_combine_kernel<K, IO>), dim3(grid_for(batch << (p - 2))),
                       dim3(MP_BLOCK), 0, st, io, (const float2*)(first ? cur : oth),
                       (const float2*)cur, logn, batch, p);
  }
  void combine(int K, int p, bool first) {
    switch (K) {
      case 1: combine_k<1>(p, first); break;
      case 2: combine_k<2>(p, first); break;
      case 3: combine_k<3>(p, first); break;
      case 4: combine_k<4>(p, first); break;
      case 5: combine_k<5>(p, first); break;
      default: err = hipErrorInvalidValue; break;
    }
  }
};

// `lv`: most forward rounds, backward rounds and chain levels per global
// pass (1 .. 5 each; a plan's schedules offer several splits); `seg`: log2
// of the LDS segment, 12 or 13.
template <class IO>
hipError_t run_multipass(const IO& io, int log2n, int64_t batch, const float* sec, float2* W0,
                         float2* W1, MpLevels lv, int seg, hipStream_t st) {
  if ((seg != 12 && seg != 13) || log2n < seg + 3 || log2n > 24 || batch < 1 ||
      (batch << (log2n - 1 - seg)) > 0x7fffffff)
    return hipErrorInvalidValue;
  if (lv.fwd < 1 || lv.fwd > 5 || lv.bwd < 1 || lv.bwd > 5 || lv.chain < 1 || lv.chain > 5)
    return hipErrorInvalidValue;
  GpuMultipass<IO> ex{io, log2n, batch, sec, W0, W1, seg, st};
  multipass_schedule(ex, log2n, seg, lv);
  if (ex.err != hipSuccess) return ex.err;
  return hipGetLastError();
}

}  // namespace

template <int DT>
hipError_t launch_multipass(bool swap, const void* in, void* out, int log2n, int64_t batch,
                            const float* sec, float2* W0, float2* W1, MpLevels lv, int seg,
                            hipStream_t st) {
  using E = typename Store<DT>::T;
  if (swap)
    return run_multipass(ContigRtIO<DT, true>((const E*)in, (E*)out, log2n), log2n, batch, sec,
                         W0, W1, lv, seg, st);
  return run_multipass(ContigRtIO<DT, false>((const E*)in, (E*)out, log2n), log2n, batch, sec,
                       W0, W1, lv, seg, st);
}

template <int DT>
hipError_t launch_multipass_real(int kind, const RealArgs& a, int log2n, int64_t rows,
                                 const float* sec, float2* W0, float2* W1, hipStream_t st) {
  using R = typename RStore<DT>::T;
  using E = typename Store<DT>::T;
  const int64_t slots = (rows + 1) / 2;
  if (kind == 0)
    return run_multipass(RealPairIO<DT, 0>{(const R*)a.in0, (E*)a.out0, rows, log2n}, log2n,
                         slots, sec, W0, W1, MpLevels{}, kMpSegLog2, st);
  return run_multipass(DctDstIO<DT, 0>{(const R*)a.in0, (const R*)a.in1, (R*)a.out0,
                                       (R*)a.out1, rows, log2n},
                       log2n, slots, sec, W0, W1, MpLevels{}, kMpSegLog2, st);
}

template hipError_t launch_multipass<QFT_MP_DT>(bool, const void*, void*, int, int64_t,
                                                const float*, float2*, float2*, MpLevels,
                                                int, hipStream_t);
template hipError_t launch_multipass_real<QFT_MP_DT>(int, const RealArgs&, int, int64_t,
                                                     const float*, float2*, float2*,
                                                     hipStream_t);

}  // namespace qftk
