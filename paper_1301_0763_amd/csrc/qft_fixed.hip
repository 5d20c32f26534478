// Fixed-point improved-QFT kernels (qft_fixed.hpp): one workgroup per
// transform, heap buffers in LDS for N <= 2^12, else in the plan's scratch.
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

template <bool SWAP, bool LDS>
__global__ __launch_bounds__(256) void fixed_kernel(const int2* x, int2* X, int logn,
                                                    const int* H, const int* shift,
                                                    int2* scratch) {
  __shared__ int2 lds[LDS ? 2 << kFxLdsLog2 : 1];
  const int64_t t = blockIdx.x;
  const int64_t N = (int64_t)1 << logn;
  int2* b0 = LDS ? lds : scratch + 2 * N * t;
  int2* b1 = b0 + N;
  fx::transform(SwapIn<SWAP>{x + N * t}, SwapOut<SWAP>{X + N * t}, b0, b1, logn,
                fx::Table{H, shift}, (int)threadIdx.x, (int)blockDim.x, DevSync{});
}

}  // namespace

hipError_t launch_fixed(bool swap, const void* in, void* out, int log2n, int64_t batch,
                        const int* H, const int* shift, int2* scratch, hipStream_t st) {
  if (log2n < 1 || log2n > kFixedMaxLog2 || batch < 1 || batch > 0x7fffffff)
    return hipErrorInvalidValue;
  if (log2n > kFxLdsLog2 && !scratch) return hipErrorInvalidValue;
  const int threads = log2n <= 9 ? 64 : 256;
  const dim3 grid((unsigned)batch), block((unsigned)threads);
  const int2* x = (const int2*)in;
  int2* X = (int2*)out;
  if (log2n <= kFxLdsLog2) {
    if (swap)
      hipLaunchKernelGGL((fixed_kernel<true, true>), grid, block, 0, st, x, X, log2n, H, shift,
                         scratch);
    else
      hipLaunchKernelGGL((fixed_kernel<false, true>), grid, block, 0, st, x, X, log2n, H, shift,
                         scratch);
  } else {
    if (swap)
      hipLaunchKernelGGL((fixed_kernel<true, false>), grid, block, 0, st, x, X, log2n, H, shift,
                         scratch);
    else
      hipLaunchKernelGGL((fixed_kernel<false, false>), grid, block, 0, st, x, X, log2n, H,
                         shift, scratch);
  }
  return hipGetLastError();
}

}  // namespace qftk
