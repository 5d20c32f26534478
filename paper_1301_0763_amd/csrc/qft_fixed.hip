// Fixed-point improved-QFT kernels (qft_fixed.hpp): heap buffers in LDS for
// N <= 2^12 (2^12 / N transforms per workgroup, each taken by its own group
// of threads), else one workgroup per transform with the buffers in the
// plan's scratch.
#include "qft_kernels.hpp"
#include "qft_fixed.hpp"

namespace qftk {
namespace {

// Input and output of the adjoint: F^H g = swap(F swap(g)), swap(a + ib) =
// b + ia, on the integer pairs (exact).
template <bool SWAP>
struct SwapIn {
  const int2* p;
  __device__ __forceinline__ int2 operator[](int64_t i) const {
    const int2 v = p[i];
    return SWAP ? make_int2(v.y, v.x) : v;
  }
};
template <bool SWAP>
struct SwapOut {
  int2* p;
  struct Ref {
    int2* q;
    __device__ __forceinline__ Ref& operator=(int2 v) {
      *q = SWAP ? make_int2(v.y, v.x) : v;
      return *this;
    }
  };
  __device__ __forceinline__ Ref operator[](int64_t i) const { return Ref{p + i}; }
};

constexpr int kFxLdsLog2 = 12;  // heap buffers of up to 2^12 cells in LDS

// Transforms per workgroup (T) and threads per transform (G): a round has
// about N/4 items (closed quads), so G = N/4 threads (64 .. 1024) keep every
// thread busy; in LDS the workgroup holds T = 2^12 / N transforms (at most
// 1024) and G shrinks so that T G <= 1024.
struct FxShape {
  int T, G;
};
inline FxShape fixed_shape(int log2n) {
  const int q = log2n >= 2 ? 1 << (log2n - 2) : 1;
  int G = q < 64 ? 64 : (q > 1024 ? 1024 : q);
  int T = 1;
  if (log2n < kFxLdsLog2) {
    T = 1 << (kFxLdsLog2 - log2n);
    if (T > 1024) T = 1024;
    if (T * G > 1024) G = 1024 / T;
  }
  return FxShape{T, G};
}

// Workgroup b: transforms b T .. b T + T - 1, transform k of them taken by
// threads k G .. k G + G - 1 (G a power of two, so a group of at most 64
// threads lies in one wavefront).  A group past the batch runs every pass with
// no items (thread index N, beyond every pass's item count, which is at most
// N), so that it meets the workgroup's barriers.
template <bool SWAP, bool LDS>
__global__ __launch_bounds__(1024) void fixed_kernel(const int2* x, int2* X, int logn,
                                                    int64_t batch, int T, const int* H,
                                                    const int* shift, int2* scratch) {
  __shared__ int2 lds[LDS ? 2 << kFxLdsLog2 : 1];
  const int G = (int)blockDim.x / T;
  const int k = (int)threadIdx.x / G, lt = (int)threadIdx.x - k * G;
  const int64_t t = (int64_t)blockIdx.x * T + k;
  const int64_t N = (int64_t)1 << logn;
  int2* b0 = LDS ? lds + 2 * N * k : scratch + 2 * N * t;
  int2* b1 = b0 + N;
  const int tt = t < batch ? lt : (int)N;
  // two forward rounds per pass from N = 2^12 on (measured faster there,
  // slower for the smaller transforms, whose passes then have too few items)
  const bool fuse2 = logn >= 12;
  // G <= 64 (N <= 2^8): each transform's threads and LDS buffers belong to
  // one wavefront, so its passes are ordered by the wavefront alone
  if (LDS && G <= kWave)
    fx::transform(SwapIn<SWAP>{x + N * t}, SwapOut<SWAP>{X + N * t}, b0, b1, logn,
                  fx::Table{H, shift}, tt, G, DevWaveSync{}, fuse2);
  else
    fx::transform(SwapIn<SWAP>{x + N * t}, SwapOut<SWAP>{X + N * t}, b0, b1, logn,
                  fx::Table{H, shift}, tt, G, DevSync{}, fuse2);
}

}  // namespace

hipError_t launch_fixed(bool swap, const void* in, void* out, int log2n, int64_t batch,
                        const int* H, const int* shift, int2* scratch, hipStream_t st) {
  if (log2n < 1 || log2n > kFixedMaxLog2 || batch < 1 || batch > 0x7fffffff)
    return hipErrorInvalidValue;
  if (log2n > kFxLdsLog2 && !scratch) return hipErrorInvalidValue;
  const FxShape sh = fixed_shape(log2n);
  const dim3 grid((unsigned)((batch + sh.T - 1) / sh.T)), block((unsigned)(sh.T * sh.G));
  const int2* x = (const int2*)in;
  int2* X = (int2*)out;
  if (log2n <= kFxLdsLog2) {
    if (swap)
      hipLaunchKernelGGL((fixed_kernel<true, true>), grid, block, 0, st, x, X, log2n, batch,
                         sh.T, H, shift, scratch);
    else
      hipLaunchKernelGGL((fixed_kernel<false, true>), grid, block, 0, st, x, X, log2n, batch,
                         sh.T, H, shift, scratch);
  } else {
    if (swap)
      hipLaunchKernelGGL((fixed_kernel<true, false>), grid, block, 0, st, x, X, log2n, batch,
                         sh.T, H, shift, scratch);
    else
      hipLaunchKernelGGL((fixed_kernel<false, false>), grid, block, 0, st, x, X, log2n, batch,
                         sh.T, H, shift, scratch);
  }
  return hipGetLastError();
}

}  // namespace qftk
