// Improved-QFT DFT library for gfx950: kernels, plans and the C ABI of
// include/qft.h.  The cell layout and the formula of every step are in
// qft_device.hpp.
//
// Execution paths
//  * tile kernel (N <= 2^14): one workgroup holds T = 2^TILE / N whole
//    transforms in LDS and runs fold -> forward rounds -> backward rounds ->
//    DCT-0/DST-0 chain -> combine, reading and writing HBM once.
//  * persistent uneven kernel: the same per-tile work over a size-sorted work
//    list of tiles (each tile = transforms of one size), grid = resident
//    workgroups, static striding (every workgroup exits after its last tile).
//  * multi-pass path (N > 2^14): fold into a global heap buffer, forward
//    rounds of the blocks larger than one 2^12-cell segment in global
//    memory, one LDS pass per segment (the core pass closes the small end of
//    the chain), backward rounds and chain levels of the large blocks in
//    global memory (ping-pong buffers for the backward rounds), combine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "qft_device.hpp"
#include "qft_schedule.hpp"
#include "../../include/qft.h"

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
#ifndef QFT_PAD
#define QFT_PAD 3
#endif
constexpr int kPad = QFT_PAD;  // LDS padding: one spare cell per 2^kPad cells

// Specialised tile kernel: T = 2^(TILE_LOG2 - LOGN) transforms of 2^LOGN.
template <int LOGN, int TILE_LOG2, int BLOCK, int DT, bool SWAP>
__global__ __launch_bounds__(BLOCK) void tile_kernel_s(const typename Store<DT>::T* x,
                                                        typename Store<DT>::T* X, int64_t batch,
                                                        const float* sec) {
  constexpr int T = 1 << (TILE_LOG2 - LOGN);
  __shared__ float2 Wl[padded_cells<kPad>(1 << TILE_LOG2)];
  const PadPtr<kPad> W{Wl, 0};
  const int64_t t0 = (int64_t)blockIdx.x * T;
  const int Tact = (int)min((int64_t)T, batch - t0);
  const int64_t off = t0 << LOGN;
  tile_body_s<DT, SWAP, LOGN, T, BLOCK, kWave>(x + off, X + off, W, Tact, sec, (int)threadIdx.x,
                                               DevSync{}, DevWaveSync{});
}

// Persistent kernel for uneven plans: tiles[w] = (logn, first, count, 0)
// covers transforms with element offsets offs[first .. first+count).
// Workgroups stride over the size-sorted list and exit after their last tile.
template <int TILE_LOG2, int BLOCK, int DT, bool SWAP>
__global__ __launch_bounds__(BLOCK) void uneven_kernel(const typename Store<DT>::T* x,
                                                        typename Store<DT>::T* X,
                                                        const int4* __restrict__ tiles,
                                                        int ntiles,
                                                        const int64_t* __restrict__ offs,
                                                        const float* sec) {
  __shared__ float2 Wl[padded_cells<kPad>(1 << TILE_LOG2)];
  const PadPtr<kPad> W{Wl, 0};
  constexpr int CPT = (1 << TILE_LOG2) / BLOCK;
  for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const int4 d = tiles[w];
    tile_body<DT, SWAP, CPT>(x, X, W, d.x, d.z, offs + d.y, sec, (int)threadIdx.x, BLOCK, kWave,
                             DevSync{}, DevWaveSync{});
    __syncthreads();
  }
}

constexpr int MP_BLOCK = 256;

#define QFT_GRID_STRIDE(i, total)                                              \
  for (int64_t i = (int64_t)blockIdx.x * MP_BLOCK + threadIdx.x; i < (total); \
       i += (int64_t)gridDim.x * MP_BLOCK)

template <int DT, bool SWAP>
__global__ __launch_bounds__(MP_BLOCK) void mp_fold_kernel(const typename Store<DT>::T* x,
                                                           float2* W, int logn, int64_t batch) {
  QFT_GRID_STRIDE(i, batch << (logn - 1)) mp_fold_item<DT, SWAP>(x, W, logn, i);
}

template <int DT, bool SWAP>
__global__ __launch_bounds__(MP_BLOCK) void mp_combine_kernel(const float2* W,
                                                              typename Store<DT>::T* X,
                                                              int logn, int64_t batch) {
  QFT_GRID_STRIDE(i, batch << (logn - 1)) mp_combine_item<DT, SWAP>(W, X, logn, i);
}

template <int K>
__global__ __launch_bounds__(MP_BLOCK) void mp_fwd_kernel(float2* W, int logn, int64_t batch,
                                                          int hi, const float* sec) {
  QFT_GRID_STRIDE(i, (2 * batch) << (logn - K - 2)) mp_fwd_item<K>(W, logn, hi, sec, i);
}

__global__ __launch_bounds__(MP_BLOCK) void mp_bwd_kernel(const float2* Win, float2* Wout,
                                                          int logn, int64_t batch, int s) {
  QFT_GRID_STRIDE(i, (2 * batch) << (logn - 2)) mp_bwd_item(Win, Wout, logn, s, i);
}

__global__ __launch_bounds__(MP_BLOCK) void mp_chain_kernel(float2* W, int logn, int64_t batch,
                                                            int p) {
  QFT_GRID_STRIDE(i, batch * chain_groups(p)) mp_chain_item(W, logn, p, i);
}

#undef QFT_GRID_STRIDE

template <int MC_LOG2, int BLOCK>
__global__ __launch_bounds__(BLOCK) void mp_segment_kernel(float2* W, int logn,
                                                           const float* sec) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int CPT = (2 * MC) / BLOCK;
  __shared__ float2 Ll[padded_cells<kPad>(2 * MC)];
  const PadPtr<kPad> L{Ll, 0};
  const int per_t = mp_segment_blocks(logn, MC_LOG2);
  const int64_t t = blockIdx.x / per_t;
  const int r = (int)(blockIdx.x - t * per_t);
  mp_segment_body<MC_LOG2, CPT>(W + (t << logn), L, logn, r, sec, (int)threadIdx.x, BLOCK, kWave,
                                DevSync{}, DevWaveSync{});
}

// Two-pass path, N = 8 * 2^MC_LOG2.  Pass A: 8 workgroups per transform
// (side x segment).  Block b serves transform 8*(b/64) + b%8 and workgroup
// role (b/8)%8, so that the eight workgroups of a transform share b%8, i.e.
// land on the same XCD (round-robin dispatch) and find x in that XCD's L2.
template <int MC_LOG2, int BLOCK, int DT, bool SWAP>
__global__ __launch_bounds__(BLOCK) void tp_a_kernel(const typename Store<DT>::T* x, float2* W,
                                                      int64_t batch, const float* sec) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int logn = MC_LOG2 + 3;
  __shared__ float2 Ll[padded_cells<kPad>(MC + 1)];
  const PadPtr<kPad> L{Ll, 0};
  const int64_t b = blockIdx.x;
  const int r = (int)(b & 63);
  const int64_t t = (b >> 6) * 8 + (r & 7);
  if (t >= batch) return;
  tp_pass_a<DT, SWAP, MC_LOG2, BLOCK>(x + (t << logn), W + (t << logn), L, r >> 3, sec,
                                      (int)threadIdx.x, kWave, DevSync{}, DevWaveSync{});
}

// Pass A with both sides per workgroup: 4 workgroups per transform, block b
// serves transform 8*(b/32) + b%8 and segment (b/8)%4 (same XCD per transform).
template <int MC_LOG2, int BLOCK, int DT, bool SWAP>
__global__ __launch_bounds__(BLOCK) void tp_a2_kernel(const typename Store<DT>::T* x, float2* W,
                                                       int64_t batch, const float* sec) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int logn = MC_LOG2 + 3;
  __shared__ float2 Ll[padded_cells<kPad>(2 * MC + 1)];
  const PadPtr<kPad> L{Ll, 0};
  const int64_t b = blockIdx.x;
  const int r = (int)(b & 31);
  const int64_t t = (b >> 5) * 8 + (r & 7);
  if (t >= batch) return;
  tp_pass_a2<DT, SWAP, MC_LOG2, BLOCK>(x + (t << logn), W + (t << logn), L, r >> 3, sec,
                                       (int)threadIdx.x, kWave, DevSync{}, DevWaveSync{});
}

template <int MC_LOG2, int DT, bool SWAP>
__global__ __launch_bounds__(256) void tp_b_kernel(const float2* W, typename Store<DT>::T* X,
                                                   int64_t batch) {
  constexpr int logn = MC_LOG2 + 3;
  const int64_t total = batch << (logn - 3);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t t = i >> (logn - 3);
    const int k = (int)(i & ((1 << (logn - 3)) - 1));
    tp_pass_b<DT, SWAP, MC_LOG2>(W + (t << logn), X + (t << logn), k);
  }
}

}  // namespace qftk

// ===========================================================================
// Host side: plans and the C ABI.
// ===========================================================================
namespace {

thread_local int g_last_hip_error = 0;

constexpr int kMaxTileLog2 = 14;  // single-workgroup transforms
constexpr int kSegLog2 = 12;      // multi-pass segment size
constexpr int kUnevenTileLog2 = 14;
constexpr int kUnevenBlock = 1024;

struct LargeItem {
  int log2n;
  int64_t offset;  // element offset
};

}  // namespace

struct qft_plan_s {
  int device = 0;
  qft_dtype dtype = QFT_C32;
  bool uneven = false;
  int log2n = 0;        // uniform plans
  int64_t batch = 0;    // uniform plans
  int64_t total_points = 0;
  double flops_5nlogn = 0.0;
  double flops_actual = 0.0;
  int max_log2n = 0;
  float* d_sec = nullptr;
  float2* d_work = nullptr;  // 2 buffers for the multi-pass path
  int64_t work_cells = 0;    // cells per buffer
  // uneven
  int4* d_tiles = nullptr;
  int ntiles = 0;
  int64_t* d_offs = nullptr;
  int persistent_grid = 0;
  std::vector<LargeItem> large;
};

namespace {

qft_status hip_fail(hipError_t e) {
  g_last_hip_error = (int)e;
  return QFT_ERROR_HIP;
}

#define QFT_HIP(call)                              \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_);     \
  } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess) {
      ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

qft_status check_device(int device) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e);
  if (device < 0 || device >= count) return QFT_ERROR_INVALID_VALUE;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e);
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return QFT_ERROR_UNSUPPORTED;
  return QFT_SUCCESS;
}

void add_costs(qft_plan_s* p, int log2n, int64_t count) {
  const double N = (double)((int64_t)1 << log2n);
  p->total_points += ((int64_t)1 << log2n) * count;
  p->flops_5nlogn += 5.0 * N * log2n * (double)count;
  p->flops_actual += (4.0 * N * log2n - 6.0 * N + 8.0) * (double)count;
}

void free_plan(qft_plan_s* p) {
  if (!p) return;
  if (p->d_sec) (void)hipFree(p->d_sec);
  if (p->d_work) (void)hipFree(p->d_work);
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  if (p->d_offs) (void)hipFree(p->d_offs);
  delete p;
}

qft_status alloc_common(qft_plan_s* p) {
  const int lg = std::max(p->max_log2n, 3);
  const int64_t nt = ((int64_t)1 << lg) / 4;
  std::vector<float> h(nt);
  qftk::fill_secants(h.data(), lg);
  QFT_HIP(hipMalloc(&p->d_sec, nt * sizeof(float)));
  QFT_HIP(hipMemcpy(p->d_sec, h.data(), nt * sizeof(float), hipMemcpyHostToDevice));
  if (p->work_cells > 0) {
    hipError_t e = hipMalloc(&p->d_work, 2 * p->work_cells * sizeof(float2));
    if (e != hipSuccess) {
      g_last_hip_error = (int)e;
      return QFT_ERROR_ALLOC;
    }
  }
  return QFT_SUCCESS;
}

inline unsigned grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  const int64_t cap = 1 << 20;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <int LOGN, int DT, bool SWAP>
void launch_tile_s(const void* in, void* out, int64_t batch, const float* sec, hipStream_t st) {
  using T = typename qftk::Store<DT>::T;
  constexpr int TL = LOGN <= 12 ? 12 : LOGN;
  constexpr int BLOCK = TL == 12 ? 256 : (TL == 13 ? 512 : 1024);
  constexpr int64_t Tmax = (int64_t)1 << (TL - LOGN);
  const int64_t grid = (batch + Tmax - 1) / Tmax;
  hipLaunchKernelGGL((qftk::tile_kernel_s<LOGN, TL, BLOCK, DT, SWAP>), dim3((unsigned)grid),
                     dim3(BLOCK), 0, st, (const T*)in, (T*)out, batch, sec);
}

template <int DT, bool SWAP>
qft_status launch_tile(const void* in, void* out, int log2n, int64_t batch, const float* sec,
                       hipStream_t st) {
  const int tl = log2n <= 12 ? 12 : log2n;
  if (((batch + ((int64_t)1 << (tl - log2n)) - 1) >> (tl - log2n)) > 0x7fffffff)
    return QFT_ERROR_INVALID_VALUE;
  switch (log2n) {
#define QFT_TILE_CASE(L) \
  case L: launch_tile_s<L, DT, SWAP>(in, out, batch, sec, st); break;
    QFT_TILE_CASE(1) QFT_TILE_CASE(2) QFT_TILE_CASE(3) QFT_TILE_CASE(4) QFT_TILE_CASE(5)
    QFT_TILE_CASE(6) QFT_TILE_CASE(7) QFT_TILE_CASE(8) QFT_TILE_CASE(9) QFT_TILE_CASE(10)
    QFT_TILE_CASE(11) QFT_TILE_CASE(12) QFT_TILE_CASE(13) QFT_TILE_CASE(14)
#undef QFT_TILE_CASE
    default: return QFT_ERROR_INVALID_SIZE;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
}

// GPU executor of the multi-pass schedule (qft_schedule.hpp).
template <int DT, bool SWAP>
struct GpuMultipass {
  using T = typename qftk::Store<DT>::T;
  const T* x;
  T* X;
  int logn;
  int64_t batch;
  const float* sec;
  float2* cur;
  float2* oth;
  hipStream_t st;
  unsigned g_elem() const { return grid_for(batch << (logn - 1), qftk::MP_BLOCK); }
  void fold() {
    hipLaunchKernelGGL((qftk::mp_fold_kernel<DT, SWAP>), dim3(g_elem()), dim3(qftk::MP_BLOCK), 0,
                       st, x, cur, logn, batch);
  }
  void fwd(int K, int hi) {
    const unsigned g = grid_for((2 * batch) << (logn - K - 2), qftk::MP_BLOCK);
    if (K == 3)
      hipLaunchKernelGGL((qftk::mp_fwd_kernel<3>), dim3(g), dim3(qftk::MP_BLOCK), 0, st, cur, logn,
                         batch, hi, sec);
    else if (K == 2)
      hipLaunchKernelGGL((qftk::mp_fwd_kernel<2>), dim3(g), dim3(qftk::MP_BLOCK), 0, st, cur, logn,
                         batch, hi, sec);
    else
      hipLaunchKernelGGL((qftk::mp_fwd_kernel<1>), dim3(g), dim3(qftk::MP_BLOCK), 0, st, cur, logn,
                         batch, hi, sec);
  }
  void segment() {
    const int64_t blocks = batch * qftk::mp_segment_blocks(logn, kSegLog2);
    hipLaunchKernelGGL((qftk::mp_segment_kernel<kSegLog2, 256>), dim3((unsigned)blocks), dim3(256),
                       0, st, cur, logn, sec);
  }
  void bwd(int s) {
    hipLaunchKernelGGL(qftk::mp_bwd_kernel, dim3(g_elem()), dim3(qftk::MP_BLOCK), 0, st,
                       (const float2*)cur, oth, logn, batch, s);
    std::swap(cur, oth);
  }
  void chain(int p) {
    hipLaunchKernelGGL(qftk::mp_chain_kernel,
                       dim3(grid_for(batch * qftk::chain_groups(p), qftk::MP_BLOCK)),
                       dim3(qftk::MP_BLOCK), 0, st, cur, logn, batch, p);
  }
  void combine() {
    hipLaunchKernelGGL((qftk::mp_combine_kernel<DT, SWAP>), dim3(g_elem()), dim3(qftk::MP_BLOCK),
                       0, st, (const float2*)cur, X, logn, batch);
  }
};

template <int DT, bool SWAP>
qft_status launch_multipass(const void* in, void* out, int log2n, int64_t batch,
                            const float* sec, float2* W0, float2* W1, hipStream_t st) {
  using T = typename qftk::Store<DT>::T;
  if (batch * qftk::mp_segment_blocks(log2n, kSegLog2) > 0x7fffffff) return QFT_ERROR_INVALID_VALUE;
  GpuMultipass<DT, SWAP> ex{(const T*)in, (T*)out, log2n, batch, sec, W0, W1, st};
  qftk::multipass_schedule(ex, log2n, kSegLog2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
}

// Two-pass path (N = 2^15, 2^16): pass A into the heap buffer W, pass B to X.
template <int DT, bool SWAP>
qft_status launch_twopass(const void* in, void* out, int log2n, int64_t batch, const float* sec,
                          float2* W, hipStream_t st) {
  using T = typename qftk::Store<DT>::T;
  const T* x = (const T*)in;
  T* X = (T*)out;
  const int64_t blocks_a = ((batch + 7) / 8) * 64;
  if (blocks_a > 0x7fffffff) return QFT_ERROR_INVALID_VALUE;
  const unsigned gb = grid_for(batch << (log2n - 3), 256);
  if (log2n == 16) {
    hipLaunchKernelGGL((qftk::tp_a2_kernel<13, 1024, DT, SWAP>), dim3((unsigned)(blocks_a / 2)),
                       dim3(1024), 0, st, x, W, batch, sec);
    hipLaunchKernelGGL((qftk::tp_b_kernel<13, DT, SWAP>), dim3(gb), dim3(256), 0, st,
                       (const float2*)W, X, batch);
  } else {
    hipLaunchKernelGGL((qftk::tp_a2_kernel<12, 512, DT, SWAP>), dim3((unsigned)(blocks_a / 2)),
                       dim3(512), 0, st, x, W, batch, sec);
    hipLaunchKernelGGL((qftk::tp_b_kernel<12, DT, SWAP>), dim3(gb), dim3(256), 0, st,
                       (const float2*)W, X, batch);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
}

// Transforms longer than one workgroup's LDS.
template <int DT, bool SWAP>
qft_status launch_large(const void* in, void* out, int log2n, int64_t batch, const float* sec,
                        float2* W0, float2* W1, hipStream_t st) {
  if (log2n == 15 || log2n == 16)
    return launch_twopass<DT, SWAP>(in, out, log2n, batch, sec, W0, st);
  return launch_multipass<DT, SWAP>(in, out, log2n, batch, sec, W0, W1, st);
}

template <int DT, bool SWAP>
qft_status launch_uneven(const qft_plan_s* p, const void* in, void* out, hipStream_t st) {
  using T = typename qftk::Store<DT>::T;
  const T* x = (const T*)in;
  T* X = (T*)out;
  if (p->ntiles > 0) {
    hipLaunchKernelGGL((qftk::uneven_kernel<kUnevenTileLog2, kUnevenBlock, DT, SWAP>),
                       dim3(p->persistent_grid), dim3(kUnevenBlock), 0, st, x, X, p->d_tiles,
                       p->ntiles, p->d_offs, p->d_sec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
  }
  for (const LargeItem& it : p->large) {
    qft_status s = launch_large<DT, SWAP>(x + it.offset, X + it.offset, it.log2n, 1, p->d_sec,
                                          p->d_work, p->d_work + p->work_cells, st);
    if (s != QFT_SUCCESS) return s;
  }
  return QFT_SUCCESS;
}

template <bool SWAP>
qft_status exec_impl(qft_plan_t plan, const void* in, void* out, void* stream) {
  if (!plan || !in || !out) return QFT_ERROR_INVALID_VALUE;
  const int64_t esz = plan->dtype == QFT_C32 ? 8 : 4;
  if (((uintptr_t)in % esz) != 0 || ((uintptr_t)out % esz) != 0) return QFT_ERROR_ALIGNMENT;
  const int64_t bytes = plan->total_points * esz;
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if (a != b && a < b + (uintptr_t)bytes && b < a + (uintptr_t)bytes) return QFT_ERROR_OVERLAP;
  DeviceGuard guard(plan->device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  hipStream_t st = (hipStream_t)stream;
  if (plan->uneven) {
    return plan->dtype == QFT_C32 ? launch_uneven<0, SWAP>(plan, in, out, st)
                                  : launch_uneven<1, SWAP>(plan, in, out, st);
  }
  if (plan->log2n <= kMaxTileLog2) {
    return plan->dtype == QFT_C32
               ? launch_tile<0, SWAP>(in, out, plan->log2n, plan->batch, plan->d_sec, st)
               : launch_tile<1, SWAP>(in, out, plan->log2n, plan->batch, plan->d_sec, st);
  }
  float2* W0 = plan->d_work;
  float2* W1 = plan->d_work + plan->work_cells;
  return plan->dtype == QFT_C32
             ? launch_large<0, SWAP>(in, out, plan->log2n, plan->batch, plan->d_sec, W0, W1, st)
             : launch_large<1, SWAP>(in, out, plan->log2n, plan->batch, plan->d_sec, W0, W1, st);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* qft_status_string(qft_status s) {
  switch (s) {
    case QFT_SUCCESS: return "success";
    case QFT_ERROR_INVALID_VALUE: return "invalid value";
    case QFT_ERROR_INVALID_SIZE: return "invalid size (log2n outside [1, 24])";
    case QFT_ERROR_ALIGNMENT: return "pointer not aligned to the element size";
    case QFT_ERROR_OVERLAP: return "input and output partially overlap";
    case QFT_ERROR_ALLOC: return "allocation failed";
    case QFT_ERROR_HIP: return "HIP runtime error";
    case QFT_ERROR_UNSUPPORTED: return "unsupported device or feature";
  }
  return "unknown status";
}

int qft_last_hip_error(void) { return g_last_hip_error; }

qft_status qft_secant_table(float* out, int log2n_max) {
  if (!out) return QFT_ERROR_INVALID_VALUE;
  if (log2n_max < 3 || log2n_max > QFT_MAX_LOG2N) return QFT_ERROR_INVALID_SIZE;
  qftk::fill_secants(out, log2n_max);
  return QFT_SUCCESS;
}

qft_status qft_plan_create(qft_plan_t* plan, int log2n, int64_t batch, qft_dtype dtype,
                           int device) {
  if (!plan) return QFT_ERROR_INVALID_VALUE;
  *plan = nullptr;
  if (batch <= 0 || (dtype != QFT_C32 && dtype != QFT_C16)) return QFT_ERROR_INVALID_VALUE;
  if (log2n < 1 || log2n > QFT_MAX_LOG2N) return QFT_ERROR_INVALID_SIZE;
  if (batch > ((int64_t)1 << 40) >> log2n) return QFT_ERROR_INVALID_VALUE;
  qft_status s = check_device(device);
  if (s != QFT_SUCCESS) return s;
  DeviceGuard guard(device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  qft_plan_s* p = new (std::nothrow) qft_plan_s();
  if (!p) return QFT_ERROR_ALLOC;
  p->device = device;
  p->dtype = dtype;
  p->log2n = log2n;
  p->batch = batch;
  p->max_log2n = log2n;
  add_costs(p, log2n, batch);
  if (log2n > kMaxTileLog2) p->work_cells = batch << log2n;
  s = alloc_common(p);
  if (s != QFT_SUCCESS) {
    free_plan(p);
    return s;
  }
  *plan = p;
  return QFT_SUCCESS;
}

qft_status qft_plan_create_uneven(qft_plan_t* plan, const int32_t* log2n, int64_t count,
                                  qft_dtype dtype, int device) {
  if (!plan) return QFT_ERROR_INVALID_VALUE;
  *plan = nullptr;
  if (!log2n || count <= 0 || (dtype != QFT_C32 && dtype != QFT_C16))
    return QFT_ERROR_INVALID_VALUE;
  if (count > (1 << 30)) return QFT_ERROR_INVALID_VALUE;
  for (int64_t i = 0; i < count; ++i)
    if (log2n[i] < 1 || log2n[i] > QFT_MAX_LOG2N) return QFT_ERROR_INVALID_SIZE;
  qft_status s = check_device(device);
  if (s != QFT_SUCCESS) return s;
  DeviceGuard guard(device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  qft_plan_s* p = new (std::nothrow) qft_plan_s();
  if (!p) return QFT_ERROR_ALLOC;
  p->device = device;
  p->dtype = dtype;
  p->uneven = true;
  for (int64_t i = 0; i < count; ++i) {
    p->max_log2n = std::max(p->max_log2n, (int)log2n[i]);
    add_costs(p, log2n[i], 1);
  }
  if (p->total_points > ((int64_t)1 << 40)) {
    free_plan(p);
    return QFT_ERROR_INVALID_VALUE;
  }
  std::vector<int64_t> off, perm, large_idx;
  std::vector<qftk::TileDesc> tdesc;
  qftk::build_uneven_worklist(log2n, count, kUnevenTileLog2, off, tdesc, perm, large_idx);
  std::vector<int4> tiles;
  for (const qftk::TileDesc& d : tdesc) tiles.push_back(make_int4(d.log2n, d.first, d.count, 0));
  int64_t large_max = 0;
  for (int64_t i : large_idx) {
    p->large.push_back({log2n[i], off[i]});
    large_max = std::max<int64_t>(large_max, (int64_t)1 << log2n[i]);
  }
  p->work_cells = large_max;
  s = alloc_common(p);
  if (s == QFT_SUCCESS && !tiles.empty()) {
    p->ntiles = (int)tiles.size();
    hipError_t e = hipMalloc(&p->d_tiles, tiles.size() * sizeof(int4));
    if (e == hipSuccess) e = hipMalloc(&p->d_offs, perm.size() * sizeof(int64_t));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_offs, perm.data(), perm.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) s = hip_fail(e);
    int cus = 0;
    if (s == QFT_SUCCESS) {
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
      if (e != hipSuccess) s = hip_fail(e);
    }
    // one 128 KiB-LDS workgroup fits per CU
    p->persistent_grid = std::max(1, std::min(p->ntiles, cus));
  }
  if (s != QFT_SUCCESS) {
    free_plan(p);
    return s;
  }
  *plan = p;
  return QFT_SUCCESS;
}

qft_status qft_exec_fwd(qft_plan_t plan, const void* in, void* out, void* stream) {
  return exec_impl<false>(plan, in, out, stream);
}

qft_status qft_exec_bwd(qft_plan_t plan, const void* in, void* out, void* stream) {
  return exec_impl<true>(plan, in, out, stream);
}

qft_status qft_plan_destroy(qft_plan_t plan) {
  if (!plan) return QFT_SUCCESS;
  DeviceGuard guard(plan->device);
  free_plan(plan);
  return QFT_SUCCESS;
}

qft_status qft_plan_info(qft_plan_t plan, int64_t* total_points, int64_t* algo_bytes,
                         double* flops_5nlogn, double* flops_actual) {
  if (!plan) return QFT_ERROR_INVALID_VALUE;
  const int64_t esz = plan->dtype == QFT_C32 ? 8 : 4;
  if (total_points) *total_points = plan->total_points;
  if (algo_bytes) *algo_bytes = 2 * plan->total_points * esz;
  if (flops_5nlogn) *flops_5nlogn = plan->flops_5nlogn;
  if (flops_actual) *flops_actual = plan->flops_actual;
  return QFT_SUCCESS;
}

}  // extern "C"
