// Improved-QFT DFT library for gfx950: plans, schedules, the two-pass
// kernels, and the C ABI of include/qft.h.  The cell layout and the formula
// of every step are in qft_device.hpp; the persistent tile kernels (N <=
// 2^14) are in qft_tiles.hip, the multi-pass path in qft_multipass.hip.
//
// Execution paths
//  * persistent tile kernel (N <= 2^14): a workgroup holds whole transforms
//    in LDS (tiles of 2^12, 2^13 or 2^14 cells) and runs fold -> forward
//    rounds -> backward rounds -> fused DCT-0/DST-0 chain and combine,
//    reading and writing HBM once; workgroups stride over a list of tiles.
//  * two-pass path (N = 2^15, 2^16): pass A gathers each quarter of a
//    transform's heap (both sides) from x and runs its rounds in LDS, pass B
//    streams the top backward round, the last two chain levels and the
//    combine.
//  * multi-pass path (N > 2^16): fold into a global heap buffer, forward
//    rounds of the blocks larger than one 2^12-cell segment (up to five per
//    pass, in registers), one LDS pass per segment, backward rounds and
//    chain levels of the large blocks (up to five per pass), the last chain
//    pass writing X.
// A plan holds one or more schedules (which transform sizes run in which
// tile-size group); qft_plan_autotune times them and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qft_cache.hpp"
#include "qft_fixed.hpp"
#include "qft_kernels.hpp"
#include "qft_schedule.hpp"
#include "../../include/qft.h"

namespace qftk {

// Two-pass path, N = 8 * 2^MC_LOG2.  Pass A: both sides of one segment per
// workgroup, 4 tiles per transform (tp_tile_transform / tp_tile_segment put
// the four on one XCD); a grid smaller than the tile count is persistent,
// its workgroups striding over the tiles (tp_pass_a2_loop).
template <int MC_LOG2, int BLOCK, int DT, bool SWAP>
__global__ __launch_bounds__(BLOCK) void tp_a2_kernel(const typename Store<DT>::T* x, float2* W,
                                                       int64_t batch, int64_t ntiles,
                                                       const float* sec) {
  constexpr int MC = 1 << MC_LOG2;
  __shared__ float2 Ll[padded_cells<kPad>(2 * MC + 1)];
  const PadPtr<kPad> L{Ll, 0};
  tp_pass_a2_loop<DT, SWAP, MC_LOG2, BLOCK, kWave>(x, W, L, batch, ntiles, (int64_t)blockIdx.x,
                                                   (int64_t)gridDim.x, sec, (int)threadIdx.x,
                                                   DevSync{}, DevWaveSync{});
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

// Static scratch of qft_exec_fwd_static (no allocation): the constant table
// of transforms up to 2^kStaticMaxLog2 (kStaticTabCells cells hold its
// floats) followed by the two-pass heap buffer.  One copy per GPU, held until
// the process ends.
constexpr int kStaticMaxLog2 = 16;
constexpr int64_t kStaticTabCells = ((int64_t)1 << kStaticMaxLog2) / 8;  // 2^14 floats
constexpr int64_t kStaticCells = (int64_t)8 << 20;                      // 64 MiB
__device__ __align__(256) float2 scratch[kStaticCells];

// Constant table entries [0, nt) computed on the device in FP64 by the same
// expression as fill_secants, rounded once to FP32.
__global__ __launch_bounds__(256) void static_secants_kernel(float* tab, int nt) {
  const int i = (int)(blockIdx.x * 256 + threadIdx.x);
  if (i >= nt) return;
  if (i == 0) {
    tab[0] = 0.0f;
    return;
  }
  const int L = 1 << (31 - __clz(i));
  const int m = i - L;
  const double a = M_PI * (double)(2 * L - 2 * m - 1) / (double)(4 * L);
  tab[i] = (float)(1.0 / (2.0 * sin(a)));
}

}  // namespace qftk

// ===========================================================================
// Host side: plans and the C ABI.
// ===========================================================================
namespace {

thread_local int g_last_hip_error = 0;

// Transforms handled outside the tile groups (N > 2^14): `batch` contiguous
// transforms of 2^log2n points starting at element `offset`.
struct LargeItem {
  int log2n;
  int64_t offset;
  int64_t batch;
};
// Most cells of one workspace buffer that an uneven plan spends on batching
// a run of same-size long transforms (2^22 cells: 32 MiB).
constexpr int64_t kLargeRunCells = (int64_t)1 << 22;

// A schedule: tile-group launches, in order, for the transforms of N <= 2^14,
// and how pass A of the two-pass path (N = 2^15, 2^16) covers its tiles.
struct Schedule {
  std::string name;
  std::vector<qftk::TileGroup> groups;
  bool tp_persistent = true;  // two-pass pass A: resident grid, else one workgroup per tile
  qftk::MpLevels mp{};        // multi-pass: most rounds / levels per global pass
  int mp_seg = qftk::kMpSegLog2;  // multi-pass: log2 of the LDS segment
};

}  // namespace

struct qft_plan_s {
  int device = 0;
  qft_dtype dtype = QFT_C32;
  bool uneven = false;
  bool real = false;          // real-input plan (rdft, DCT-0/DST-0)
  int64_t real_algo_bytes = 0;
  int log2n = 0;        // uniform plans
  int64_t batch = 0;    // uniform plans
  int64_t total_points = 0;
  double flops_5nlogn = 0.0;
  double flops_actual = 0.0;
  int max_log2n = 0;
  int cus = 0;
  float* d_sec = nullptr;
  float2* d_work = nullptr;  // heap buffers of the two-pass / multi-pass paths
  int64_t work_cells = 0;    // cells per buffer
  int work_buffers = 0;      // 1 (two-pass only) or 2 (multi-pass)
  int64_t tp_resident[2] = {0, 0};  // pass-A workgroups resident at once, N = 2^15, 2^16
  std::vector<Schedule> schedules;
  int chosen = 0;
  std::vector<LargeItem> large;  // common to every schedule
  std::vector<void*> dev_allocs;  // tile lists of the groups (shared between schedules)
  bool fixed = false;              // QFT_I32 plan: the fixed-point transform
  int* d_fxH = nullptr;            // its integer constant table (N/4 mantissas)
  int* d_fxShift = nullptr;        // and the shift of each slice
  std::string cache_key;          // schedule-cache key (device and plan shape)
  bool from_cache = false;        // the chosen schedule came from the cache
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

qft_status check_device(int device, int* cus) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e);
  if (device < 0 || device >= count) return QFT_ERROR_INVALID_VALUE;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e);
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return QFT_ERROR_UNSUPPORTED;
  *cus = prop.multiProcessorCount;
  return QFT_SUCCESS;
}

// Schedule-cache key: the device (gfx950 and its CU count) and the plan's
// shape; uneven plans are identified by a 64-bit FNV-1a hash of their sizes.
std::string plan_key(const qft_plan_s* p, const char* kind, const int32_t* sizes,
                     int64_t count) {
  std::string k = "gfx950/" + std::to_string(p->cus) + "cu/" + kind + "/" +
                  (p->dtype == QFT_C32 ? "c32" : p->dtype == QFT_C16 ? "c16" : "i32") + "/";
  if (sizes) {
    uint64_t h = 1469598103934665603ull;
    for (int64_t i = 0; i < count; ++i) {
      h ^= (uint64_t)(uint32_t)sizes[i];
      h *= 1099511628211ull;
    }
    char buf[40];
    std::snprintf(buf, sizeof buf, "%lld:%016llx", (long long)count, (unsigned long long)h);
    return k + buf;
  }
  return k + std::to_string(p->log2n) + "x" + std::to_string(p->batch);
}

// Starts the plan on the schedule the cache names for its key, if any.
void apply_cached_schedule(qft_plan_s* p) {
  std::string name;
  if (!qftk::schedule_cache_lookup(qftk::schedule_cache_path(), p->cache_key, name)) return;
  for (size_t i = 0; i < p->schedules.size(); ++i) {
    if (p->schedules[i].name == name) {
      p->chosen = (int)i;
      p->from_cache = true;
      return;
    }
  }
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
  if (p->d_fxH) (void)hipFree(p->d_fxH);
  if (p->d_fxShift) (void)hipFree(p->d_fxShift);
  for (void* a : p->dev_allocs) (void)hipFree(a);
  delete p;
}

qft_status alloc_common(qft_plan_s* p) {
  // at least the table of 2^14 points: the persistent tile kernel of 2^TL-cell
  // tiles copies the first 2^TL / 4 floats into LDS whatever sizes it runs
  const int lg = std::max(p->max_log2n, qftk::kMaxTileLog2);
  const int64_t nt = ((int64_t)1 << lg) / 4;
  std::vector<float> h(nt);
  qftk::fill_secants(h.data(), lg);
  QFT_HIP(hipMalloc(&p->d_sec, nt * sizeof(float)));
  QFT_HIP(hipMemcpy(p->d_sec, h.data(), nt * sizeof(float), hipMemcpyHostToDevice));
  if (p->work_cells > 0) {
    hipError_t e = hipMalloc(&p->d_work, p->work_buffers * p->work_cells * sizeof(float2));
    if (e != hipSuccess) {
      g_last_hip_error = (int)e;
      return QFT_ERROR_ALLOC;
    }
  }
  return QFT_SUCCESS;
}

// Grid of a tile group: the resident workgroups (persistent: each strides
// over the tiles) or one workgroup per tile (the hardware dispatcher hands
// out tiles as workgroups finish).
int group_grid(const qft_plan_s* p, int tl, int64_t ntiles, bool persistent) {
  const int64_t cap = (int64_t)std::max(p->cus, 1) * qftk::tile_wgs_per_cu(tl);
  return (int)std::max<int64_t>(1, persistent ? std::min<int64_t>(ntiles, cap) : ntiles);
}

// Uniform batch of N = 2^log2n <= 2^tl in tiles of 2^tl cells.
qft_status uniform_group(const qft_plan_s* p, int tl, qftk::TileGroup* g) {
  const int64_t per = (int64_t)1 << (tl - p->log2n);
  const int64_t ntiles = (p->batch + per - 1) / per;
  if (ntiles > 0x7fffffff) return QFT_ERROR_INVALID_VALUE;
  *g = qftk::TileGroup{tl, (int)ntiles, (int)ntiles, nullptr, nullptr, p->log2n, p->batch, 0};
  return QFT_SUCCESS;
}

// Uneven transforms with lo <= log2n <= hi in tiles of 2^tl cells.
qft_status uneven_group(qft_plan_s* p, const int32_t* log2n, const std::vector<int64_t>& offsets,
                        int lo, int hi, int tl, qftk::TileGroup* g) {
  std::vector<qftk::TileDesc> desc;
  std::vector<int64_t> perm;
  qftk::build_tiles(log2n, offsets, lo, hi, tl, desc, perm);
  *g = qftk::TileGroup{tl, (int)desc.size(), group_grid(p, tl, (int64_t)desc.size(), true),
                       nullptr, nullptr, 0, 0, 0};
  g->single_log2n = lo == hi ? lo : 0;
  if (desc.empty()) return QFT_SUCCESS;
  std::vector<int4> tiles;
  for (const qftk::TileDesc& d : desc) tiles.push_back(make_int4(d.log2n, d.first, d.count, 0));
  QFT_HIP(hipMalloc(&g->d_tiles, tiles.size() * sizeof(int4)));
  p->dev_allocs.push_back(g->d_tiles);
  QFT_HIP(hipMalloc(&g->d_offs, perm.size() * sizeof(int64_t)));
  p->dev_allocs.push_back(g->d_offs);
  QFT_HIP(hipMemcpy(g->d_tiles, tiles.data(), tiles.size() * sizeof(int4),
                    hipMemcpyHostToDevice));
  QFT_HIP(hipMemcpy(g->d_offs, perm.data(), perm.size() * sizeof(int64_t),
                    hipMemcpyHostToDevice));
  return QFT_SUCCESS;
}

inline unsigned grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  const int64_t cap = 1 << 20;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Two-pass path (N = 2^15, 2^16): pass A into the heap buffer W, pass B to X.
// `resident` is the number of pass-A workgroups the device holds at once
// (0: one workgroup per tile, no persistence).
template <int DT, bool SWAP>
qft_status launch_twopass(const void* in, void* out, int log2n, int64_t batch, const float* sec,
                          float2* W, int64_t resident, hipStream_t st) {
  using T = typename qftk::Store<DT>::T;
  const T* x = (const T*)in;
  T* X = (T*)out;
  const int64_t ntiles = ((batch + 7) / 8) * 32;
  if (ntiles > 0x7fffffff) return QFT_ERROR_INVALID_VALUE;
  int64_t grid_a = ntiles;
  if (resident > 0 && resident < ntiles)  // persistent; whole groups of 32 keep j per workgroup
    grid_a = resident >= 32 ? resident / 32 * 32 : resident;
  const unsigned gb = grid_for(batch << (log2n - 3), 256);
  if (log2n == 16) {
    hipLaunchKernelGGL((qftk::tp_a2_kernel<13, qftk::kTpBlock13, DT, SWAP>), dim3((unsigned)grid_a),
                       dim3(qftk::kTpBlock13), 0, st, x, W, batch, ntiles, sec);
    hipLaunchKernelGGL((qftk::tp_b_kernel<13, DT, SWAP>), dim3(gb), dim3(256), 0, st,
                       (const float2*)W, X, batch);
  } else {
    hipLaunchKernelGGL((qftk::tp_a2_kernel<12, 256, DT, SWAP>), dim3((unsigned)grid_a),
                       dim3(256), 0, st, x, W, batch, ntiles, sec);
    hipLaunchKernelGGL((qftk::tp_b_kernel<12, DT, SWAP>), dim3(gb), dim3(256), 0, st,
                       (const float2*)W, X, batch);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
}

// Transforms longer than one workgroup's LDS.
template <int DT, bool SWAP>
qft_status launch_large(const qft_plan_s* p, const Schedule& s, const void* in, void* out,
                        int log2n, int64_t batch, float2* W0, float2* W1, hipStream_t st) {
  const float* sec = p->d_sec;
  if (log2n == 15 || log2n == 16)
    return launch_twopass<DT, SWAP>(in, out, log2n, batch, sec, W0,
                                    s.tp_persistent ? p->tp_resident[log2n - 15] : 0, st);
  const hipError_t e =
      qftk::launch_multipass<DT>(SWAP, in, out, log2n, batch, sec, W0, W1, s.mp, s.mp_seg, st);
  return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
}

template <int DT, bool SWAP>
qft_status run_schedule(const qft_plan_s* p, const Schedule& s, const void* in, void* out,
                        hipStream_t st) {
  using E = typename qftk::Store<DT>::T;
  for (const qftk::TileGroup& g : s.groups) {
    if (g.ntiles == 0) continue;
    hipError_t e = hipErrorInvalidValue;
    switch (g.tl) {
      case 10: e = qftk::launch_tiles<DT, 10, SWAP>(g, in, out, p->d_sec, st); break;
      case 11: e = qftk::launch_tiles<DT, 11, SWAP>(g, in, out, p->d_sec, st); break;
      case 12: e = qftk::launch_tiles<DT, 12, SWAP>(g, in, out, p->d_sec, st); break;
      case 13: e = qftk::launch_tiles<DT, 13, SWAP>(g, in, out, p->d_sec, st); break;
      case 14: e = qftk::launch_tiles<DT, 14, SWAP>(g, in, out, p->d_sec, st); break;
      default: break;
    }
    if (e != hipSuccess) return hip_fail(e);
  }
  float2* W0 = p->d_work;
  float2* W1 = p->work_buffers > 1 ? p->d_work + p->work_cells : nullptr;
  for (const LargeItem& it : p->large) {
    const qft_status r = launch_large<DT, SWAP>(p, s, (const E*)in + it.offset,
                                                (E*)out + it.offset, it.log2n, it.batch, W0, W1,
                                                st);
    if (r != QFT_SUCCESS) return r;
  }
  return QFT_SUCCESS;
}

// Bytes of one complex element of the plan's storage type.
int64_t elem_size(qft_dtype dt) { return dt == QFT_C16 ? 4 : 8; }

qft_status check_buffers(const qft_plan_s* plan, const void* in, const void* out) {
  if (!plan || !in || !out) return QFT_ERROR_INVALID_VALUE;
  const int64_t esz = elem_size(plan->dtype);
  if (((uintptr_t)in % esz) != 0 || ((uintptr_t)out % esz) != 0) return QFT_ERROR_ALIGNMENT;
  const int64_t bytes = plan->total_points * esz;
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if (a != b && a < b + (uintptr_t)bytes && b < a + (uintptr_t)bytes) return QFT_ERROR_OVERLAP;
  return QFT_SUCCESS;
}

template <bool SWAP>
qft_status exec_sched(const qft_plan_s* plan, int sched, const void* in, void* out,
                      hipStream_t st) {
  if (plan->fixed) {
    const hipError_t e = qftk::launch_fixed(SWAP, in, out, plan->log2n, plan->batch,
                                            plan->d_fxH, plan->d_fxShift, (int2*)plan->d_work,
                                            st);
    return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
  }
  const Schedule& s = plan->schedules[sched];
  return plan->dtype == QFT_C32 ? run_schedule<0, SWAP>(plan, s, in, out, st)
                                : run_schedule<1, SWAP>(plan, s, in, out, st);
}

template <bool SWAP>
qft_status exec_impl(qft_plan_t plan, const void* in, void* out, void* stream) {
  if (plan && plan->real) return QFT_ERROR_INVALID_VALUE;
  const qft_status c = check_buffers(plan, in, out);
  if (c != QFT_SUCCESS) return c;
  DeviceGuard guard(plan->device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  return exec_sched<SWAP>(plan, plan->chosen, in, out, (hipStream_t)stream);
}

// The fixed-point plan (QFT_I32): integer constant table and, for N > 2^12,
// two heap buffers of N int2 cells per transform.
qft_status create_fixed(qft_plan_s* p) {
  const int lg = std::max(p->log2n, 3);
  const int64_t nt = ((int64_t)1 << lg) / 4;
  std::vector<int> H((size_t)nt), shift(32, 0);
  qftk::fx::fill_table_q(H.data(), shift.data(), lg);
  QFT_HIP(hipMalloc(&p->d_fxH, nt * sizeof(int)));
  QFT_HIP(hipMemcpy(p->d_fxH, H.data(), nt * sizeof(int), hipMemcpyHostToDevice));
  QFT_HIP(hipMalloc(&p->d_fxShift, shift.size() * sizeof(int)));
  QFT_HIP(hipMemcpy(p->d_fxShift, shift.data(), shift.size() * sizeof(int),
                    hipMemcpyHostToDevice));
  if (p->log2n > 12) {
    const int64_t bytes = 2 * (p->batch << p->log2n) * (int64_t)sizeof(int2);
    hipError_t e = hipMalloc(&p->d_work, bytes);
    if (e != hipSuccess) {
      g_last_hip_error = (int)e;
      return QFT_ERROR_ALLOC;
    }
  }
  p->schedules.push_back(Schedule{"fixed", {}, true, {}});
  return QFT_SUCCESS;
}

// Byte range [p, p + n) of a real-input exec argument; null pointers are empty.
struct Span {
  uintptr_t a = 0, b = 0;
  Span(const void* p, int64_t n) : a((uintptr_t)p), b(p ? (uintptr_t)p + (uintptr_t)n : 0) {}
  bool overlaps(const Span& o) const { return a && o.a && a < o.b && o.a < b; }
};

qft_status run_real(const qft_plan_s* p, int kind, const qftk::RealArgs& a, hipStream_t st) {
  if (p->log2n > qftk::kMaxTileLog2) {
    float2* W0 = p->d_work;
    float2* W1 = p->d_work + p->work_cells;
    const hipError_t e =
        p->dtype == QFT_C16
            ? qftk::launch_multipass_real<1>(kind, a, p->log2n, p->batch, p->d_sec, W0, W1, st)
            : qftk::launch_multipass_real<0>(kind, a, p->log2n, p->batch, p->d_sec, W0, W1, st);
    return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
  }
  const qftk::TileGroup& g = p->schedules[p->chosen].groups[0];
  hipError_t e = hipErrorInvalidValue;
  const bool h16 = p->dtype == QFT_C16;
  switch (g.tl) {
    case 10: e = h16 ? qftk::launch_real<1, 10>(g, kind, a, p->d_sec, st)
                     : qftk::launch_real<0, 10>(g, kind, a, p->d_sec, st); break;
    case 11: e = h16 ? qftk::launch_real<1, 11>(g, kind, a, p->d_sec, st)
                     : qftk::launch_real<0, 11>(g, kind, a, p->d_sec, st); break;
    case 12: e = h16 ? qftk::launch_real<1, 12>(g, kind, a, p->d_sec, st)
                     : qftk::launch_real<0, 12>(g, kind, a, p->d_sec, st); break;
    case 13: e = h16 ? qftk::launch_real<1, 13>(g, kind, a, p->d_sec, st)
                     : qftk::launch_real<0, 13>(g, kind, a, p->d_sec, st); break;
    case 14: e = h16 ? qftk::launch_real<1, 14>(g, kind, a, p->d_sec, st)
                     : qftk::launch_real<0, 14>(g, kind, a, p->d_sec, st); break;
    default: break;
  }
  return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
}

// Pass-A workgroups the device holds at once (resident grid of the
// persistent two-pass launch); 0 if the occupancy query fails, which makes
// the launch fall back to one workgroup per tile.
template <int DT>
void set_tp_resident_dt(qft_plan_s* p) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&qftk::tp_a2_kernel<12, 256, DT, false>), 256, 0) ==
          hipSuccess && nb > 0)
    p->tp_resident[0] = (int64_t)nb * p->cus;
  nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&qftk::tp_a2_kernel<13, qftk::kTpBlock13, DT, false>),
          qftk::kTpBlock13, 0) ==
          hipSuccess && nb > 0)
    p->tp_resident[1] = (int64_t)nb * p->cus;
  (void)hipGetLastError();
}

void set_tp_resident(qft_plan_s* p) {
  if (p->dtype == QFT_C16) set_tp_resident_dt<1>(p);
  else set_tp_resident_dt<0>(p);
}

qft_plan_s* new_plan(int device, qft_dtype dtype, int cus) {
  qft_plan_s* p = new (std::nothrow) qft_plan_s();
  if (p) {
    p->device = device;
    p->dtype = dtype;
    p->cus = cus;
  }
  return p;
}

// Per-device state of qft_exec_fwd_static: the address of that device's copy
// of qftk::scratch (hipGetSymbolAddress; the symbol's own name is a host
// stand-in that must never reach a kernel) and the resident pass-A grids.
struct StaticDev {
  std::once_flag once;
  hipError_t err = hipSuccess;
  float2* ptr = nullptr;
  int64_t tp_resident[2] = {0, 0};
};
constexpr int kMaxDevices = 64;
StaticDev g_static[kMaxDevices];

qft_status static_setup(int dev, StaticDev** out) {
  if (dev < 0 || dev >= kMaxDevices) return QFT_ERROR_UNSUPPORTED;
  StaticDev& d = g_static[dev];
  std::call_once(d.once, [&d, dev]() {
    d.err = hipGetSymbolAddress((void**)&d.ptr, HIP_SYMBOL(qftk::scratch));
    if (d.err != hipSuccess) {
      d.ptr = nullptr;
      return;
    }
    qft_plan_s probe;  // plan fields the occupancy query reads, no allocation
    probe.device = dev;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
      probe.cus = cus;
      set_tp_resident(&probe);
      d.tp_resident[0] = probe.tp_resident[0];
      d.tp_resident[1] = probe.tp_resident[1];
    }
    (void)hipGetLastError();
  });
  if (d.err != hipSuccess || !d.ptr) return hip_fail(d.err != hipSuccess ? d.err
                                                                         : hipErrorInvalidSymbol);
  *out = &d;
  return QFT_SUCCESS;
}

template <int DT>
qft_status static_exec(const StaticDev& d, int log2n, int64_t batch, const void* in, void* out,
                       hipStream_t st) {
  float* tab = reinterpret_cast<float*>(d.ptr);
  const int nt = (1 << std::max(log2n, 3)) / 4;
  hipLaunchKernelGGL(qftk::static_secants_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256),
                     0, st, tab, nt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  if (log2n <= qftk::kMaxTileLog2) {
    const int tl = std::max(qftk::kMinTileLog2, log2n);
    const int64_t per = (int64_t)1 << (tl - log2n);
    const int64_t ntiles = (batch + per - 1) / per;
    if (ntiles > 0x7fffffff) return QFT_ERROR_INVALID_VALUE;
    const qftk::TileGroup g{tl, (int)ntiles, (int)ntiles, nullptr, nullptr, log2n, batch, 0};
    switch (tl) {
      case 10: e = qftk::launch_tiles<DT, 10, false>(g, in, out, tab, st); break;
      case 11: e = qftk::launch_tiles<DT, 11, false>(g, in, out, tab, st); break;
      case 12: e = qftk::launch_tiles<DT, 12, false>(g, in, out, tab, st); break;
      case 13: e = qftk::launch_tiles<DT, 13, false>(g, in, out, tab, st); break;
      default: e = qftk::launch_tiles<DT, 14, false>(g, in, out, tab, st); break;
    }
    return e == hipSuccess ? QFT_SUCCESS : hip_fail(e);
  }
  return launch_twopass<DT, false>(in, out, log2n, batch, tab, d.ptr + qftk::kStaticTabCells,
                                   d.tp_resident[log2n - 15], st);
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
    case QFT_ERROR_SCRATCH:
      return "request exceeds the static scratch of qft_exec_fwd_static "
             "(log2n <= 16; batch * 2^log2n <= 8M - 16K points for log2n = 15, 16)";
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
  if (batch <= 0 || (dtype != QFT_C32 && dtype != QFT_C16 && dtype != QFT_I32))
    return QFT_ERROR_INVALID_VALUE;
  if (log2n < 1 || log2n > QFT_MAX_LOG2N) return QFT_ERROR_INVALID_SIZE;
  if (dtype == QFT_I32 && log2n > qftk::kFixedMaxLog2) return QFT_ERROR_INVALID_SIZE;
  if (batch > ((int64_t)1 << 40) >> log2n) return QFT_ERROR_INVALID_VALUE;
  if (dtype == QFT_I32 && batch > 0x7fffffff) return QFT_ERROR_INVALID_VALUE;
  int cus = 0;
  qft_status s = check_device(device, &cus);
  if (s != QFT_SUCCESS) return s;
  DeviceGuard guard(device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  qft_plan_s* p = new_plan(device, dtype, cus);
  if (!p) return QFT_ERROR_ALLOC;
  p->log2n = log2n;
  p->batch = batch;
  p->max_log2n = log2n;
  add_costs(p, log2n, batch);
  if (dtype == QFT_I32) {
    p->fixed = true;
    s = create_fixed(p);
    if (s != QFT_SUCCESS) {
      free_plan(p);
      return s;
    }
    *plan = p;
    return QFT_SUCCESS;
  }
  if (log2n <= qftk::kMaxTileLog2) {
    // schedule 0: the kernel specialised for this size, one workgroup per
    // tile of 2^max(10, log2n) cells
    const int tl = std::max(qftk::kMinTileLog2, log2n);
    Schedule sc;
    sc.name = "t" + std::to_string(tl) + ":" + std::to_string(log2n);
    sc.groups.resize(1);
    s = uniform_group(p, tl, &sc.groups[0]);
    if (s == QFT_SUCCESS) p->schedules.push_back(sc);
    // the same with the constant table copied into LDS; and for one
    // transform of 2^13 or 2^14 points per tile on a resident grid that
    // loads each next tile during the current one, where there are more
    // tiles than resident workgroups
    if (s == QFT_SUCCESS) {
      Schedule ls = sc;
      ls.name += "/lds";
      ls.groups[0].lds_sec = true;
      p->schedules.push_back(ls);
      Schedule pp = ls;
      pp.name = sc.name + "/pipe";
      pp.groups[0].grid = group_grid(p, tl, pp.groups[0].ntiles, true);
      if (log2n >= 13 && pp.groups[0].grid < pp.groups[0].ntiles) p->schedules.push_back(pp);
    }
    // the size-generic persistent kernel of uneven plans on a transform list,
    // tiles of 2^tl2 cells for every tl2 that holds a transform (batches of
    // at most 2^20 transforms: the list costs 8 bytes per transform)
    if (batch <= ((int64_t)1 << 20)) {
      std::vector<int32_t> sizes((size_t)batch, log2n);
      std::vector<int64_t> off;
      qftk::packed_offsets(sizes.data(), batch, off);
      for (int tl2 = tl; tl2 <= qftk::kMaxTileLog2 && s == QFT_SUCCESS; ++tl2) {
        Schedule g;
        g.name = "g" + std::to_string(tl2) + ":" + std::to_string(log2n);
        g.groups.resize(1);
        s = uneven_group(p, sizes.data(), off, log2n, log2n, tl2, &g.groups[0]);
        if (s == QFT_SUCCESS) p->schedules.push_back(g);
      }
    }
  } else {
    p->work_cells = batch << log2n;
    p->work_buffers = log2n <= 16 ? 1 : 2;
    p->large.push_back({log2n, 0, batch});
    if (log2n <= 16) {
      p->schedules.push_back(Schedule{"two-pass", {}, true, {}});
      p->schedules.push_back(Schedule{"two-pass/all", {}, false, {}});
    } else {
      // splits of the global passes: most forward rounds / backward rounds /
      // chain levels per pass, with LDS segments of 2^12 cells and, as
      // "/s13", of 2^13 (one round and one chain level fewer in the global
      // passes, one workgroup per CU in the segment pass); the first is the
      // default
      const int splits[][3] = {{4, 5, 5}, {3, 5, 5}, {4, 4, 5}, {4, 5, 4}, {3, 4, 4}, {5, 5, 5}};
      for (const int seg : {12, 13}) {
        if (log2n < seg + 3) continue;
        for (const auto& sp : splits) {
          Schedule m{"multi-pass:" + std::to_string(sp[0]) + "," + std::to_string(sp[1]) + "," +
                         std::to_string(sp[2]) + (seg == 13 ? "/s13" : ""),
                     {}, true, qftk::MpLevels{sp[0], sp[1], sp[2]}, seg};
          p->schedules.push_back(m);
        }
      }
    }
    set_tp_resident(p);
  }
  if (s == QFT_SUCCESS) s = alloc_common(p);
  if (s != QFT_SUCCESS) {
    free_plan(p);
    return s;
  }
  p->cache_key = plan_key(p, "u", nullptr, 0);
  apply_cached_schedule(p);
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
  int cus = 0;
  qft_status s = check_device(device, &cus);
  if (s != QFT_SUCCESS) return s;
  DeviceGuard guard(device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  qft_plan_s* p = new_plan(device, dtype, cus);
  if (!p) return QFT_ERROR_ALLOC;
  p->uneven = true;
  bool has[QFT_MAX_LOG2N + 1] = {};
  for (int64_t i = 0; i < count; ++i) {
    p->max_log2n = std::max(p->max_log2n, (int)log2n[i]);
    has[log2n[i]] = true;
    add_costs(p, log2n[i], 1);
  }
  if (p->total_points > ((int64_t)1 << 40)) {
    free_plan(p);
    return QFT_ERROR_INVALID_VALUE;
  }
  std::vector<int64_t> off;
  qftk::packed_offsets(log2n, count, off);
  // transforms beyond one workgroup, largest first
  std::vector<int64_t> big;
  for (int64_t i = 0; i < count; ++i)
    if (log2n[i] > qftk::kMaxTileLog2) big.push_back(i);
  std::stable_sort(big.begin(), big.end(),
                   [&](int64_t a, int64_t b) { return log2n[a] > log2n[b]; });
  // a run of same-size transforms that lie back to back in memory is one
  // batched launch (its workspace at most kLargeRunCells per buffer)
  for (size_t a = 0; a < big.size();) {
    const int lg = log2n[big[a]];
    const int64_t cap = std::max<int64_t>(1, kLargeRunCells >> lg);
    int64_t k = 1;
    while (a + k < big.size() && k < cap && log2n[big[a + k]] == lg &&
           off[big[a + k]] == off[big[a]] + (k << lg))
      ++k;
    p->large.push_back({lg, off[big[a]], k});
    p->work_cells = std::max<int64_t>(p->work_cells, k << lg);
    p->work_buffers = std::max(p->work_buffers, lg <= 16 ? 1 : 2);
    a += (size_t)k;
  }
  if (!big.empty()) set_tp_resident(p);
  // Candidate schedules: tile size for N <= 2^10, 2^11, 2^12, 2^13 and 2^14;
  // sizes with the same tile size share one launch.  Each comes with a
  // resident (persistent) grid and, as "<name>/all", with one workgroup per
  // tile.  The first one runs every N <= 2^14 in a single persistent launch.
  constexpr int kCand = 7;
  const int cand[kCand][5] = {{14, 14, 14, 14, 14}, {13, 13, 13, 13, 14}, {12, 12, 12, 14, 14},
                              {12, 12, 12, 13, 14}, {10, 11, 12, 13, 14}, {10, 11, 12, 14, 14},
                              {10, 12, 12, 13, 14}};
  std::vector<Schedule> persistent;
  for (int c = 0; c < kCand && s == QFT_SUCCESS; ++c) {
    int tl_of[qftk::kMaxTileLog2 + 1];
    for (int r = 1; r <= qftk::kMaxTileLog2; ++r)
      tl_of[r] = cand[c][r <= 10 ? 0 : r - 10];
    // launches: maximal runs of present sizes with the same tile size
    std::vector<int> lo_hi;
    std::string name;
    for (int r = 1; r <= qftk::kMaxTileLog2; ++r) {
      if (!has[r]) continue;
      if (!lo_hi.empty() && tl_of[lo_hi[lo_hi.size() - 2]] == tl_of[r]) {
        lo_hi.back() = r;
      } else {
        lo_hi.push_back(r);
        lo_hi.push_back(r);
      }
    }
    for (size_t k = 0; k < lo_hi.size(); k += 2) {
      const int lo = lo_hi[k], hi = lo_hi[k + 1];
      if (!name.empty()) name += "+";
      name += "t" + std::to_string(tl_of[lo]) + ":" + std::to_string(lo) +
              (hi > lo ? "-" + std::to_string(hi) : "");
    }
    if (name.empty()) name = "large-only";
    bool dup = false;
    for (const Schedule& o : persistent) dup |= o.name == name;
    if (dup) continue;
    Schedule sc;
    sc.name = name;
    for (size_t k = 0; k < lo_hi.size() && s == QFT_SUCCESS; k += 2) {
      qftk::TileGroup g{};
      s = uneven_group(p, log2n, off, lo_hi[k], lo_hi[k + 1], tl_of[lo_hi[k]], &g);
      sc.groups.push_back(g);
    }
    persistent.push_back(sc);
  }
  for (const Schedule& sc : persistent) p->schedules.push_back(sc);
  for (const Schedule& sc : persistent) {
    if (sc.groups.empty()) continue;
    Schedule all = sc;
    all.name += "/all";
    for (qftk::TileGroup& g : all.groups) g.grid = std::max(g.ntiles, 1);
    p->schedules.push_back(all);
  }
  // "/pipe": the groups that hold only transforms of 2^13 or 2^14 points (one
  // per tile) run on a resident grid that loads each next tile during the
  // current one, where they have more tiles than resident workgroups
  for (const Schedule& sc : persistent) {
    Schedule pp = sc;
    bool any = false;
    for (qftk::TileGroup& g : pp.groups) {
      if (g.single_log2n == g.tl && g.tl >= 13 && g.ntiles > g.grid) {
        g.pipe = true;
        any = true;
      }
    }
    if (!any) continue;
    pp.name += "/pipe";
    p->schedules.push_back(pp);
  }
  if (s == QFT_SUCCESS) s = alloc_common(p);
  if (s != QFT_SUCCESS) {
    free_plan(p);
    return s;
  }
  p->cache_key = plan_key(p, "v", log2n, count);
  apply_cached_schedule(p);
  *plan = p;
  return QFT_SUCCESS;
}

qft_status qft_exec_fwd(qft_plan_t plan, const void* in, void* out, void* stream) {
  return exec_impl<false>(plan, in, out, stream);
}

qft_status qft_exec_fwd_static(int log2n, int64_t batch, qft_dtype dtype, const void* in,
                               void* out, void* stream) {
  if (!in || !out || batch <= 0 || (dtype != QFT_C32 && dtype != QFT_C16))
    return QFT_ERROR_INVALID_VALUE;
  if (log2n < 1 || log2n > QFT_MAX_LOG2N) return QFT_ERROR_INVALID_SIZE;
  if (log2n > qftk::kStaticMaxLog2) return QFT_ERROR_SCRATCH;
  if (log2n > qftk::kMaxTileLog2 &&
      batch > (qftk::kStaticCells - qftk::kStaticTabCells) >> log2n)
    return QFT_ERROR_SCRATCH;
  if (batch > ((int64_t)1 << 40) >> log2n) return QFT_ERROR_INVALID_VALUE;
  const int64_t esz = dtype == QFT_C32 ? 8 : 4;
  if (((uintptr_t)in % esz) != 0 || ((uintptr_t)out % esz) != 0) return QFT_ERROR_ALIGNMENT;
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  const uintptr_t bytes = (uintptr_t)((batch << log2n) * esz);
  if (a != b && a < b + bytes && b < a + bytes) return QFT_ERROR_OVERLAP;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  StaticDev* d = nullptr;
  const qft_status st = static_setup(dev, &d);
  if (st != QFT_SUCCESS) return st;
  return dtype == QFT_C32 ? static_exec<0>(*d, log2n, batch, in, out, (hipStream_t)stream)
                          : static_exec<1>(*d, log2n, batch, in, out, (hipStream_t)stream);
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
  const int64_t esz = elem_size(plan->dtype);
  if (total_points) *total_points = plan->total_points;
  if (algo_bytes) *algo_bytes = plan->real ? plan->real_algo_bytes : 2 * plan->total_points * esz;
  if (flops_5nlogn) *flops_5nlogn = plan->flops_5nlogn;
  if (flops_actual) *flops_actual = plan->flops_actual;
  return QFT_SUCCESS;
}

qft_status qft_plan_schedules(qft_plan_t plan, int* count, int* chosen) {
  if (!plan) return QFT_ERROR_INVALID_VALUE;
  if (count) *count = (int)plan->schedules.size();
  if (chosen) *chosen = plan->chosen;
  return QFT_SUCCESS;
}

const char* qft_plan_schedule_name(qft_plan_t plan, int schedule) {
  if (!plan || schedule < 0 || schedule >= (int)plan->schedules.size()) return nullptr;
  return plan->schedules[schedule].name.c_str();
}

qft_status qft_plan_set_schedule(qft_plan_t plan, int schedule) {
  if (!plan || schedule < 0 || schedule >= (int)plan->schedules.size())
    return QFT_ERROR_INVALID_VALUE;
  plan->chosen = schedule;
  return QFT_SUCCESS;
}

qft_status qft_plan_autotune(qft_plan_t plan, const void* in, void* out, void* stream, int reps,
                             double* ms, int ms_len, int* chosen) {
  if (plan && plan->real) return QFT_ERROR_INVALID_VALUE;
  qft_status c = check_buffers(plan, in, out);
  if (c != QFT_SUCCESS) return c;
  if (reps < 1 || reps > 10000 || ms_len < 0 || (ms_len > 0 && !ms))
    return QFT_ERROR_INVALID_VALUE;
  DeviceGuard guard(plan->device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  QFT_HIP(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e);
  }
  int best = -1;
  float best_ms = 0.f;
  for (int i = 0; i < (int)plan->schedules.size() && c == QFT_SUCCESS; ++i) {
    c = exec_sched<false>(plan, i, in, out, st);  // warm-up
    if (c == QFT_SUCCESS) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && c == QFT_SUCCESS && e == hipSuccess; ++r)
      c = exec_sched<false>(plan, i, in, out, st);
    if (c == QFT_SUCCESS && e == hipSuccess) e = hipEventRecord(e1, st);
    if (c == QFT_SUCCESS && e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (c == QFT_SUCCESS && e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (c == QFT_SUCCESS && e != hipSuccess) c = hip_fail(e);
    if (c == QFT_SUCCESS) {
      t /= (float)reps;
      if (i < ms_len) ms[i] = t;
      if (best < 0 || t < best_ms) {
        best = i;
        best_ms = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (c != QFT_SUCCESS) return c;
  plan->chosen = best;
  plan->from_cache = false;
  if (chosen) *chosen = best;
  // remembered for later plans of this shape (best effort: a cache that
  // cannot be written only means they tune again)
  if (plan->schedules.size() > 1 && !plan->cache_key.empty())
    (void)qftk::schedule_cache_store(qftk::schedule_cache_path(), plan->cache_key,
                                     plan->schedules[best].name);
  return QFT_SUCCESS;
}

qft_status qft_plan_create_real(qft_plan_t* plan, int log2n, int64_t batch, qft_dtype dtype,
                                int device) {
  if (!plan) return QFT_ERROR_INVALID_VALUE;
  *plan = nullptr;
  if (batch <= 0 || (dtype != QFT_C32 && dtype != QFT_C16)) return QFT_ERROR_INVALID_VALUE;
  if (log2n < 1 || log2n > QFT_MAX_LOG2N) return QFT_ERROR_INVALID_SIZE;
  if (batch > ((int64_t)1 << 40) >> log2n) return QFT_ERROR_INVALID_VALUE;
  int cus = 0;
  qft_status s = check_device(device, &cus);
  if (s != QFT_SUCCESS) return s;
  DeviceGuard guard(device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  qft_plan_s* p = new_plan(device, dtype, cus);
  if (!p) return QFT_ERROR_ALLOC;
  p->real = true;
  p->log2n = log2n;
  p->batch = batch;
  p->max_log2n = log2n;
  const int64_t N = (int64_t)1 << log2n;
  const int64_t rsz = dtype == QFT_C32 ? 4 : 2;
  p->total_points = batch * N;
  p->flops_5nlogn = 2.5 * (double)N * log2n * (double)batch;
  // Table 2, RDFT row: (N log N - 3N)/2 + 2 multiplications, (3 N log N - 5N)/2 + 4 additions
  p->flops_actual = (2.0 * (double)N * log2n - 4.0 * (double)N + 6.0) * (double)batch;
  p->real_algo_bytes = batch * (N * rsz + (N / 2 + 1) * 2 * rsz);
  const int64_t slots = (batch + 1) / 2;
  if (log2n > qftk::kMaxTileLog2) {
    // multi-pass path on the transform slots, heap buffers of slots * N cells
    p->work_cells = slots << log2n;
    p->work_buffers = 2;
    p->schedules.push_back(Schedule{"multi-pass/real", {}, true});
  } else {
    const int tl = std::max(qftk::kMinTileLog2, log2n);
    const int64_t per = (int64_t)1 << (tl - log2n);
    const int64_t ntiles = (slots + per - 1) / per;
    if (ntiles > 0x7fffffff) {
      free_plan(p);
      return QFT_ERROR_INVALID_VALUE;
    }
    Schedule sc;
    sc.name = "t" + std::to_string(tl) + ":" + std::to_string(log2n) + "/real";
    sc.groups.push_back(qftk::TileGroup{tl, (int)ntiles, (int)ntiles, nullptr, nullptr, log2n,
                                        slots, batch});
    p->schedules.push_back(sc);
  }
  s = alloc_common(p);
  if (s != QFT_SUCCESS) {
    free_plan(p);
    return s;
  }
  *plan = p;
  return QFT_SUCCESS;
}

qft_status qft_exec_rdft(qft_plan_t plan, const void* in, void* out, void* stream) {
  if (!plan || !plan->real || !in || !out) return QFT_ERROR_INVALID_VALUE;
  const int64_t rsz = plan->dtype == QFT_C32 ? 4 : 2;
  if (((uintptr_t)in % rsz) != 0 || ((uintptr_t)out % (2 * rsz)) != 0) return QFT_ERROR_ALIGNMENT;
  const int64_t N = (int64_t)1 << plan->log2n;
  if (Span(in, plan->batch * N * rsz).overlaps(Span(out, plan->batch * (N / 2 + 1) * 2 * rsz)))
    return QFT_ERROR_OVERLAP;
  DeviceGuard guard(plan->device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  return run_real(plan, 0, qftk::RealArgs{in, nullptr, out, nullptr}, (hipStream_t)stream);
}

qft_status qft_exec_dct0_dst0(qft_plan_t plan, const void* c, const void* d, void* C, void* S,
                              void* stream) {
  if (!plan || !plan->real) return QFT_ERROR_INVALID_VALUE;
  const int64_t N = (int64_t)1 << plan->log2n, h = N / 2;
  if (h - 1 == 0) d = S = nullptr;  // N = 2: the DST-0 has no points
  if ((c == nullptr) != (C == nullptr) || (d == nullptr) != (S == nullptr) || (!c && !d))
    return QFT_ERROR_INVALID_VALUE;
  const int64_t rsz = plan->dtype == QFT_C32 ? 4 : 2;
  for (const void* q : {(const void*)c, (const void*)d, (const void*)C, (const void*)S})
    if (((uintptr_t)q % rsz) != 0) return QFT_ERROR_ALIGNMENT;
  const Span sc(c, plan->batch * (h + 1) * rsz), sd(d, plan->batch * (h - 1) * rsz);
  const Span sC(C, plan->batch * (h + 1) * rsz), sS(S, plan->batch * (h - 1) * rsz);
  // in place (c == C, d == S) is allowed; every other overlap is not
  if ((c != C && sc.overlaps(sC)) || (d != S && sd.overlaps(sS)) || sc.overlaps(sd) ||
      sc.overlaps(sS) || sd.overlaps(sC) || sC.overlaps(sS))
    return QFT_ERROR_OVERLAP;
  DeviceGuard guard(plan->device);
  if (!guard.ok) return hip_fail(hipErrorInvalidDevice);
  return run_real(plan, 1, qftk::RealArgs{c, d, C, S}, (hipStream_t)stream);
}

}  // extern "C"
