// CPU emulation of the improved-QFT GPU library, for tests.
//
// Runs the unchanged kernel bodies of paper_1301_0763_amd/csrc/qft_device.hpp
// and the host schedules of qft_schedule.hpp on the CPU:
//  * a workgroup is emulated by `nthr` OS threads and a std::barrier;
//  * every LDS (and heap-buffer) access goes through a tracking pointer; at
//    each barrier (and at the end of every emulated global pass) a cell that
//    was written by one thread and touched by another within the same phase
//    is counted as a race, unless both threads are lanes of one wavefront
//    (64 consecutive threads) and a wave-level sync of that wavefront lies
//    between the two accesses (its lanes are then ordered, as on the GPU).
// Entry points return the number of races found (>= 0) or a negative error.
#include <hip/hip_runtime.h>

#include <atomic>
#include <barrier>
#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <algorithm>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../paper_1301_0763_amd/csrc/qft_cache.hpp"
#include "../../paper_1301_0763_amd/csrc/qft_device.hpp"
#include "../../paper_1301_0763_amd/csrc/qft_fixed.hpp"
#include "../../paper_1301_0763_amd/csrc/qft_schedule.hpp"

namespace {

struct Entry {
  int64_t cell;
  int64_t wave;  // wavefront of the actor (a unique id per workgroup wave)
  int64_t wp;    // wave-level syncs that wavefront had passed
  int64_t actor;
  bool write;
};

struct Tracker {
  std::vector<std::vector<Entry>> logs;  // one per OS thread slot
  int64_t races = 0;
  std::atomic<int64_t> oob{0};  // accesses outside the tracked buffer
  explicit Tracker(int slots) : logs(slots) {}
  // A cell races if two different actors touched it and one of them wrote,
  // unless both belong to one wavefront and touched it in different wave
  // phases.
  void end_phase() {
    std::vector<Entry> all;
    size_t n = 0;
    for (auto& lg : logs) n += lg.size();
    all.reserve(n);
    for (auto& lg : logs) {
      all.insert(all.end(), lg.begin(), lg.end());
      lg.clear();
    }
    std::sort(all.begin(), all.end(), [](const Entry& a, const Entry& b) {
      if (a.cell != b.cell) return a.cell < b.cell;
      if (a.wave != b.wave) return a.wave < b.wave;
      return a.wp < b.wp;
    });
    for (size_t i = 0; i < all.size();) {
      size_t e = i;
      bool written = false, multi_wave = false;
      while (e < all.size() && all[e].cell == all[i].cell) {
        written |= all[e].write;
        multi_wave |= all[e].wave != all[i].wave;
        ++e;
      }
      bool race = written && multi_wave;
      for (size_t a = i; !race && a < e;) {  // one wave: phase by phase
        size_t b = a;
        bool w = false, multi_actor = false;
        while (b < e && all[b].wp == all[a].wp) {
          w |= all[b].write;
          multi_actor |= all[b].actor != all[a].actor;
          ++b;
        }
        race = w && multi_actor;
        a = b;
      }
      races += race;
      i = e;
    }
  }
};

thread_local int tl_slot = 0;       // which log this OS thread appends to
thread_local int64_t tl_actor = 0;  // emulated GPU thread / work item
thread_local int64_t tl_wave = 0;   // its wavefront
thread_local int64_t tl_wp = 0;     // wave-level syncs passed by that wavefront
std::atomic<int64_t> g_workgroups{0};

// A work item of a global pass: its own wavefront (no wave-level syncs).
inline void set_item_actor(int64_t a) {
  tl_actor = a;
  tl_wave = -1 - a;
  tl_wp = 0;
}

struct Ref {
  float2* p;
  int64_t cell;
  Tracker* tr;
  operator float2() const {
    tr->logs[tl_slot].push_back({cell, tl_wave, tl_wp, tl_actor, false});
    return *p;
  }
  Ref& operator=(float2 v) {
    tr->logs[tl_slot].push_back({cell, tl_wave, tl_wp, tl_actor, true});
    *p = v;
    return *this;
  }
  Ref& operator=(const Ref& r) { return *this = (float2)r; }
};

// Tracked pointer; with ps > 0 it applies the same padding map as the
// kernels' LDS pointer (logical cell c at c + (c >> ps)).
struct TPtr {
  float2* base;
  int64_t off;
  Tracker* tr;
  int64_t size;  // logical cells of the buffer starting at base
  int ps = 0;
  Ref operator[](int64_t i) const {
    static float2 sink;
    const int64_t c = off + i;
    if (c < 0 || c >= size) {
      tr->oob++;
      return Ref{&sink, -1, tr};
    }
    const int64_t pc = ps ? c + (c >> ps) : c;
    return Ref{base + pc, (int64_t)(uintptr_t)(base + pc), tr};
  }
  Ref operator*() const { return (*this)[0]; }
  TPtr operator+(int64_t d) const { return TPtr{base, off + d, tr, size, ps}; }
};

// Tracked int2 cells (the fixed-point path).
struct IRef {
  int2* p;
  int64_t cell;
  Tracker* tr;
  operator int2() const {
    tr->logs[tl_slot].push_back({cell, tl_wave, tl_wp, tl_actor, false});
    return *p;
  }
  IRef& operator=(int2 v) {
    tr->logs[tl_slot].push_back({cell, tl_wave, tl_wp, tl_actor, true});
    *p = v;
    return *this;
  }
  IRef& operator=(const IRef& r) { return *this = (int2)r; }
};

struct IPtr {
  int2* base;
  int64_t off;
  Tracker* tr;
  int64_t size;
  IRef operator[](int64_t i) const {
    static int2 sink;
    const int64_t c = off + i;
    if (c < 0 || c >= size) {
      tr->oob++;
      return IRef{&sink, -1, tr};
    }
    return IRef{base + c, (int64_t)(uintptr_t)(base + c), tr};
  }
  IPtr operator+(int64_t d) const { return IPtr{base, off + d, tr, size}; }
};

// Row accesses of the kernels (pad_row in qft_device.hpp) on an emulated
// buffer: the exact cell, plus a check of the condition under which the
// GPU's padded row arithmetic is exact for a padding block of up to
// kRowCells cells (offsets in whole kRowCells, runs inside one 8-cell block,
// anchors inside the buffer); an access that breaks it counts as out of
// bounds, so the test fails.
struct TRow {
  TPtr t;
  int64_t blk() const { return t.ps ? (int64_t)1 << t.ps : 0; }
  Ref operator[](int64_t k) const {
    if (blk() && (k % qftk::kRowCells) != 0) t.tr->oob++;
    return t[k];
  }
  Ref run(int64_t e) const {
    if (blk()) {
      const int64_t b = blk(), m = ((t.off % b) + b) % b;
      if (e < 0 || m + e >= b) t.tr->oob++;
    }
    return t[e];
  }
};
inline TRow pad_row(const TPtr& sd, int a) {
  if (sd.ps && sd.off + a < 0) sd.tr->oob++;  // rows are anchored inside the buffer
  return TRow{sd + a};
}

constexpr int kEmuPad = 4;  // same LDS padding as the GPU kernels

// Runs fn(tid, sync, wsync) on nthr threads sharing one barrier whose
// completion closes a tracker phase; wsync is a barrier of the thread's
// wavefront (threads 64 w .. 64 w + 63) that starts a new wave phase.
template <class F>
void run_workgroup(int nthr, Tracker& tr, F fn) {
  constexpr int kLanes = 64;
  auto done = [&tr]() noexcept { tr.end_phase(); };
  std::barrier bar(nthr, done);
  const int nw = (nthr + kLanes - 1) / kLanes;
  std::vector<std::unique_ptr<std::barrier<>>> wbar;
  for (int w = 0; w < nw; ++w)
    wbar.emplace_back(new std::barrier<>(std::min(kLanes, nthr - w * kLanes)));
  const int64_t wg = g_workgroups++;
  struct HostSync {
    decltype(bar)* b;
    void operator()() const { b->arrive_and_wait(); }
  };
  struct HostWaveSync {
    std::barrier<>* b;
    void operator()() const {
      b->arrive_and_wait();
      ++tl_wp;
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nthr; ++t) {
    th.emplace_back([&, t]() {
      tl_slot = t;
      tl_actor = t;
      tl_wave = wg * 1024 + t / kLanes;
      tl_wp = 0;
      fn(t, HostSync{&bar}, HostWaveSync{wbar[t / kLanes].get()});
    });
  }
  for (auto& x : th) x.join();
  tr.end_phase();
}


// The specialised tile kernel exactly as launched on the GPU: LOGN <= 10 uses
// 2^10-cell tiles of 64 threads, larger LOGN a tile of 2^LOGN cells.  The
// uniform kernel runs a single transform of 2^13 or 2^14 points with 32
// cells per thread, every other tile (and the uneven kernel) with 16.
template <int LOGN, int TL>
constexpr int emu_tile_threads(bool uneven) {
  return (!uneven && LOGN == TL && TL >= 13) ? (1 << TL) / 32 : (1 << TL) / 16;
}

template <int DT, bool SWAP, int LOGN, int NT>
int tile_s_run(const void* x, void* X, int Tact, const float* sec, const int64_t* offs) {
  using E = typename qftk::Store<DT>::T;
  constexpr int TL = LOGN <= 10 ? 10 : LOGN;
  constexpr int T = 1 << (TL - LOGN);
  if (Tact < 1 || Tact > T) return -2;
  const int64_t cells = (int64_t)T << LOGN;
  std::vector<float2> lds(cells + (cells >> kEmuPad));
  Tracker tr(NT);
  TPtr W{lds.data(), 0, &tr, cells, kEmuPad};
  run_workgroup(NT, tr, [&](int tid, auto sync, auto wsync) {
    if (offs) {
      const qftk::GatherIO<DT, SWAP> io((const E*)x, (E*)X, offs, LOGN);
      qftk::tile_body_s<LOGN, T, NT, 64>(io, W, Tact, sec, tid, sync, wsync);
    } else {
      // the uniform kernel: one forward code path for both sides with 16
      // cells per thread, as on the GPU
      const qftk::ContigIO<DT, SWAP, LOGN> io((const E*)x, (E*)X);
      qftk::tile_body_s<LOGN, T, NT, 64, NT == (1 << TL) / 16>(io, W, Tact, sec, tid, sync,
                                                               wsync);
    }
  });
  return tr.oob ? -100 : (int)tr.races;
}

// The resident-grid tile kernel: `grid` workgroups, workgroup b taking tiles
// b, b + grid, .. of a contiguous batch and loading each next tile's x while
// the current one runs (tile_loop_s), with the GPU's tile size and threads.
template <int DT, bool SWAP, int LOGN>
int tile_p_impl(const void* x, void* X, int64_t batch, int64_t grid, const float* sec) {
  using E = typename qftk::Store<DT>::T;
  constexpr int TL = LOGN <= 10 ? 10 : LOGN;
  constexpr int NT = emu_tile_threads<LOGN, TL>(false);
  constexpr int T = 1 << (TL - LOGN);
  const int64_t cells = (int64_t)T << LOGN;
  int64_t races = 0;
  for (int64_t b = 0; b < grid; ++b) {
    std::vector<float2> lds(cells + (cells >> kEmuPad));
    Tracker tr(NT);
    TPtr W{lds.data(), 0, &tr, cells, kEmuPad};
    run_workgroup(NT, tr, [&](int tid, auto sync, auto wsync) {
      qftk::tile_loop_s<LOGN, T, NT, 64>(qftk::ContigTiles<DT, SWAP, LOGN, T>{(const E*)x, (E*)X,
                                                                            batch},
                                        b, grid, W, sec, tid, sync, wsync, []() {});
    });
    if (tr.oob) return -100;
    races += tr.races;
  }
  return (int)races;
}

// The resident-grid kernel of an uneven group of one-transform tiles
// (tile_kernel_pg): tile w = tiles[w] = (log2n, first, 1, 0), the transform
// at element offset offs[first]; the GPU's threads for a 2^LOGN tile.
template <int DT, bool SWAP, int LOGN>
int tile_pg_impl(const void* x, void* X, const int4* tiles, const int64_t* offs, int64_t ntiles,
                 int64_t grid, const float* sec) {
  using E = typename qftk::Store<DT>::T;
  constexpr int NT = emu_tile_threads<LOGN, LOGN>(false);
  const int64_t cells = (int64_t)1 << LOGN;
  int64_t races = 0;
  for (int64_t b = 0; b < grid; ++b) {
    std::vector<float2> lds(cells + (cells >> kEmuPad));
    Tracker tr(NT);
    TPtr W{lds.data(), 0, &tr, cells, kEmuPad};
    run_workgroup(NT, tr, [&](int tid, auto sync, auto wsync) {
      qftk::tile_loop_s<LOGN, 1, NT, 64>(
          qftk::ListTiles<DT, SWAP, LOGN>{(const E*)x, (E*)X, tiles, offs, ntiles}, b, grid, W,
          sec, tid, sync, wsync, []() {});
    });
    if (tr.oob) return -100;
    races += tr.races;
  }
  return (int)races;
}

template <int DT, bool SWAP, int LOGN>
int tile_s_impl(const void* x, void* X, int Tact, const float* sec, const int64_t* offs) {
  constexpr int TL = LOGN <= 10 ? 10 : LOGN;
  if (offs) return tile_s_run<DT, SWAP, LOGN, emu_tile_threads<LOGN, TL>(true)>(x, X, Tact, sec, offs);
  return tile_s_run<DT, SWAP, LOGN, emu_tile_threads<LOGN, TL>(false)>(x, X, Tact, sec, offs);
}

// One workgroup of the real-input tile kernel: KIND 0 = rdft of `rows` real
// signals (two per transform slot), 1 = DCT-0/DST-0; rows <= 2 T.
template <int DT, int LOGN, int KIND>
int tile_real_impl(int64_t rows, const void* in0, const void* in1, void* out0, void* out1,
                   const float* sec) {
  using R = typename qftk::RStore<DT>::T;
  using E = typename qftk::Store<DT>::T;
  constexpr int TL = LOGN <= 10 ? 10 : LOGN;
  constexpr int NT = emu_tile_threads<LOGN, TL>(false);
  constexpr bool SF = NT == (1 << TL) / 16;  // as the GPU's real-input kernel
  constexpr int T = 1 << (TL - LOGN);
  const int slots = (int)((rows + 1) / 2);
  if (rows < 1 || slots > T) return -2;
  const int64_t cells = (int64_t)T << LOGN;
  std::vector<float2> lds(cells + (cells >> kEmuPad));
  Tracker tr(NT);
  TPtr W{lds.data(), 0, &tr, cells, kEmuPad};
  run_workgroup(NT, tr, [&](int tid, auto sync, auto wsync) {
    if constexpr (KIND == 0) {
      const qftk::RealPairIO<DT, LOGN> io{(const R*)in0, (E*)out0, rows};
      qftk::tile_body_s<LOGN, T, NT, 64, SF>(io, W, slots, sec, tid, sync, wsync);
    } else {
      const qftk::DctDstIO<DT, LOGN> io{(const R*)in0, (const R*)in1, (R*)out0, (R*)out1, rows};
      qftk::tile_body_s<LOGN, T, NT, 64, SF>(io, W, slots, sec, tid, sync, wsync);
    }
  });
  return tr.oob ? -100 : (int)tr.races;
}

template <int DT, int KIND>
int tile_real_dispatch(int logn, int64_t rows, const void* in0, const void* in1, void* out0,
                       void* out1, const float* sec) {
  switch (logn) {
#define QFT_EMU_REAL(L) \
  case L: return tile_real_impl<DT, L, KIND>(rows, in0, in1, out0, out1, sec);
    QFT_EMU_REAL(1) QFT_EMU_REAL(2) QFT_EMU_REAL(3) QFT_EMU_REAL(4) QFT_EMU_REAL(5)
    QFT_EMU_REAL(6) QFT_EMU_REAL(7) QFT_EMU_REAL(8) QFT_EMU_REAL(9) QFT_EMU_REAL(10)
    QFT_EMU_REAL(11) QFT_EMU_REAL(12) QFT_EMU_REAL(13) QFT_EMU_REAL(14)
#undef QFT_EMU_REAL
    default: return -1;
  }
}

template <int DT, bool SWAP>
int tile_s_dispatch(const void* x, void* X, int logn, int Tact, const float* sec,
                    const int64_t* offs) {
  switch (logn) {
    case 1: return tile_s_impl<DT, SWAP, 1>(x, X, Tact, sec, offs);
    case 2: return tile_s_impl<DT, SWAP, 2>(x, X, Tact, sec, offs);
    case 3: return tile_s_impl<DT, SWAP, 3>(x, X, Tact, sec, offs);
    case 4: return tile_s_impl<DT, SWAP, 4>(x, X, Tact, sec, offs);
    case 5: return tile_s_impl<DT, SWAP, 5>(x, X, Tact, sec, offs);
    case 6: return tile_s_impl<DT, SWAP, 6>(x, X, Tact, sec, offs);
    case 7: return tile_s_impl<DT, SWAP, 7>(x, X, Tact, sec, offs);
    case 8: return tile_s_impl<DT, SWAP, 8>(x, X, Tact, sec, offs);
    case 9: return tile_s_impl<DT, SWAP, 9>(x, X, Tact, sec, offs);
    case 10: return tile_s_impl<DT, SWAP, 10>(x, X, Tact, sec, offs);
    case 11: return tile_s_impl<DT, SWAP, 11>(x, X, Tact, sec, offs);
    case 12: return tile_s_impl<DT, SWAP, 12>(x, X, Tact, sec, offs);
    case 13: return tile_s_impl<DT, SWAP, 13>(x, X, Tact, sec, offs);
    case 14: return tile_s_impl<DT, SWAP, 14>(x, X, Tact, sec, offs);
    default: return -1;
  }
}

template <int DT, bool SWAP>
int tile_p_dispatch(const void* x, void* X, int logn, int64_t batch, int64_t grid,
                    const float* sec) {
  switch (logn) {
    case 1: return tile_p_impl<DT, SWAP, 1>(x, X, batch, grid, sec);
    case 2: return tile_p_impl<DT, SWAP, 2>(x, X, batch, grid, sec);
    case 3: return tile_p_impl<DT, SWAP, 3>(x, X, batch, grid, sec);
    case 4: return tile_p_impl<DT, SWAP, 4>(x, X, batch, grid, sec);
    case 5: return tile_p_impl<DT, SWAP, 5>(x, X, batch, grid, sec);
    case 6: return tile_p_impl<DT, SWAP, 6>(x, X, batch, grid, sec);
    case 7: return tile_p_impl<DT, SWAP, 7>(x, X, batch, grid, sec);
    case 8: return tile_p_impl<DT, SWAP, 8>(x, X, batch, grid, sec);
    case 9: return tile_p_impl<DT, SWAP, 9>(x, X, batch, grid, sec);
    case 10: return tile_p_impl<DT, SWAP, 10>(x, X, batch, grid, sec);
    case 11: return tile_p_impl<DT, SWAP, 11>(x, X, batch, grid, sec);
    case 12: return tile_p_impl<DT, SWAP, 12>(x, X, batch, grid, sec);
    case 13: return tile_p_impl<DT, SWAP, 13>(x, X, batch, grid, sec);
    case 14: return tile_p_impl<DT, SWAP, 14>(x, X, batch, grid, sec);
    default: return -1;
  }
}

std::vector<float> secants(int lg) {
  lg = lg < 3 ? 3 : lg;
  std::vector<float> s(((size_t)1 << lg) / 4);
  qftk::fill_secants(s.data(), lg);  // the library's host generator
  return s;
}

// CPU executor of the multi-pass schedule: every pass runs its work items
// one after another through the tracked pointers, one phase per pass.
template <class IO>
struct EmuMultipass {
  IO io;
  int logn;
  int64_t batch;
  int seg_log2;
  int nthr;
  const float* sec;
  float2* cur;
  float2* oth;
  int64_t cells;
  Tracker gtr{64};  // one log per emulated lane
  int64_t races = 0;
  template <class F>
  void items(int64_t total, F f) {
    tl_slot = 0;
    for (int64_t i = 0; i < total; ++i) {
      set_item_actor(i);
      f(i);
    }
    gtr.end_phase();
  }
  TPtr G(float2* p) { return TPtr{p, 0, &gtr, cells}; }
  void fold() {
    items(batch << (logn - 1), [&](int64_t i) { qftk::mp_fold_io_item(io, G(cur), logn, i); });
  }
  template <int K>
  void fwd_k(int hi) {
    items((2 * batch) << (logn - K - 2),
          [&](int64_t i) { qftk::mp_fwd_item<K>(G(cur), logn, hi, sec, i); });
  }
  void fwd(int K, int hi) {
    switch (K) {
      case 1: fwd_k<1>(hi); break;
      case 2: fwd_k<2>(hi); break;
      case 3: fwd_k<3>(hi); break;
      case 4: fwd_k<4>(hi); break;
      case 5: fwd_k<5>(hi); break;
      default: races = -1000000; break;
    }
  }
  template <int MC_LOG2>
  void segment_mc() {
    // the GPU's 32 cells per thread for 2^12- and 2^13-cell segments, else
    // <= 32 threads
    constexpr int MC = 1 << MC_LOG2;
    constexpr int NT = MC_LOG2 >= 12 ? (2 * MC) / 32 : (MC < 32 ? MC : 32);
    const int segs = 1 << (logn - 1 - MC_LOG2);
    for (int64_t b = 0; b < batch * segs; ++b) {
      const int64_t t = b / segs;
      const int j = (int)(b - t * segs);
      const int64_t lc = 2 * MC + 1;
      std::vector<float2> lds(lc + (lc >> kEmuPad));
      Tracker ltr(NT);
      TPtr L{lds.data(), 0, &ltr, lc, kEmuPad};
      float2* wt = cur + (t << logn);
      run_workgroup(NT, ltr, [&](int tid, auto sync, auto wsync) {
        qftk::mp_segment_pair<MC_LOG2, NT, 64>(wt, L, 1 << (logn - 1), j, sec, tid, sync, wsync);
      });
      races += ltr.races;
      if (ltr.oob) races = -1000000;
    }
  }
  void segment() {
    switch (seg_log2) {
      case 3: segment_mc<3>(); break;
      case 4: segment_mc<4>(); break;
      case 5: segment_mc<5>(); break;
      case 6: segment_mc<6>(); break;
      case 8: segment_mc<8>(); break;
      case 10: segment_mc<10>(); break;
      case 12: segment_mc<12>(); break;
      case 13: segment_mc<13>(); break;
      default: races = -1000000; break;
    }
  }
  template <int K>
  void bwd_k(int hi) {
    const int64_t total = (2 * batch) << (logn - 1 - K);
    if (hi - K >= 6 && logn - 1 - K >= 6) {
      // as the GPU runs it: 64-lane wavefronts staging their outputs in LDS
      constexpr int ROW = qftk::MpBwdStage<K>::ROW;
      for (int64_t w = 0; w < total / 64; ++w) {
        std::vector<float2> lds(64 * ROW);
        Tracker ltr(64);
        TPtr L{lds.data(), 0, &ltr, 64 * ROW};
        run_workgroup(64, ltr, [&](int tid, auto, auto wsync) {
          tl_actor = w * 64 + tid;  // unique over the pass
          qftk::mp_bwd_wave_item<K, 64>(G(cur), G(oth), L, logn, hi, w * 64 + tid, tid, wsync);
        });
        races += ltr.races;
        if (ltr.oob) races = -1000000;
      }
      gtr.end_phase();
    } else {
      items(total,
            [&](int64_t i) { qftk::mp_bwd_group_item<K>(G(cur), G(oth), logn, hi, i); });
    }
    std::swap(cur, oth);
  }
  void bwd(int K, int hi) {
    switch (K) {
      case 1: bwd_k<1>(hi); break;
      case 2: bwd_k<2>(hi); break;
      case 3: bwd_k<3>(hi); break;
      case 4: bwd_k<4>(hi); break;
      case 5: bwd_k<5>(hi); break;
      default: races = -1000000; break;
    }
  }
  template <int K>
  void chain_k(int p, bool first) {
    float2* e = first ? cur : oth;
    items(batch << (p - 2),
          [&](int64_t i) { qftk::mp_chain_item<K>(G(e), G(cur), G(oth), logn, p, i); });
  }
  void chain(int K, int p, bool first) {
    switch (K) {
      case 1: chain_k<1>(p, first); break;
      case 2: chain_k<2>(p, first); break;
      case 3: chain_k<3>(p, first); break;
      case 4: chain_k<4>(p, first); break;
      case 5: chain_k<5>(p, first); break;
      default: races = -1000000; break;
    }
  }
  template <int K>
  void combine_k(int p, bool first) {
    float2* e = first ? cur : oth;
    items(batch << (p - 2),
          [&](int64_t i) { qftk::mp_chain_combine_item<K>(io, G(e), G(cur), logn, p, i); });
  }
  void combine(int K, int p, bool first) {
    switch (K) {
      case 1: combine_k<1>(p, first); break;
      case 2: combine_k<2>(p, first); break;
      case 3: combine_k<3>(p, first); break;
      case 4: combine_k<4>(p, first); break;
      case 5: combine_k<5>(p, first); break;
      default: races = -1000000; break;
    }
  }
};

template <class IO>
int run_multipass(const IO& io, int logn, int64_t batch, int seg_log2, int nthr,
                  const float* sec, qftk::MpLevels lv = qftk::MpLevels{}) {
  std::vector<float2> w0((size_t)batch << logn), w1((size_t)batch << logn);
  EmuMultipass<IO> ex{io, logn, batch, seg_log2, nthr, sec, w0.data(), w1.data(),
                      (int64_t)batch << logn};
  qftk::multipass_schedule(ex, logn, seg_log2, lv);
  if (ex.races < 0 || ex.gtr.oob) return -4;
  return (int)(ex.races + ex.gtr.races);
}

template <int DT, bool SWAP>
int multipass_impl(const void* x, void* X, int logn, int64_t batch, int seg_log2, int nthr,
                   const float* sec, qftk::MpLevels lv = qftk::MpLevels{}) {
  using E = typename qftk::Store<DT>::T;
  if (logn < seg_log2 + 3) return -3;
  return run_multipass(qftk::ContigRtIO<DT, SWAP>((const E*)x, (E*)X, logn), logn, batch,
                       seg_log2, nthr, sec, lv);
}

// Multi-pass path of a real-input plan (kind 0: rdft, 1: DCT-0/DST-0).
template <int DT>
int multipass_real_impl(int kind, int logn, int64_t rows, const void* in0, const void* in1,
                        void* out0, void* out1, int seg_log2, int nthr, const float* sec) {
  using R = typename qftk::RStore<DT>::T;
  using E = typename qftk::Store<DT>::T;
  if (logn < seg_log2 + 3) return -3;
  const int64_t slots = (rows + 1) / 2;
  if (kind == 0)
    return run_multipass(qftk::RealPairIO<DT, 0>{(const R*)in0, (E*)out0, rows, logn}, logn,
                         slots, seg_log2, nthr, sec);
  return run_multipass(
      qftk::DctDstIO<DT, 0>{(const R*)in0, (const R*)in1, (R*)out0, (R*)out1, rows, logn}, logn,
      slots, seg_log2, nthr, sec);
}

// Uneven packed batch as the library runs it: transforms of up to 2^10
// points in 2^10-cell tiles of the size-sorted work list, 2^11 .. 2^14 in a
// tile of their own (the persistent kernel's larger tile sizes), all through
// the specialised tile kernel with the offset list; longer ones through the
// multi-pass schedule (segments of 2^seg_log2 cells).
template <int DT, bool SWAP>
int twopass_impl(const void* x, void* X, int mc_log2, int64_t batch, int64_t grid);

template <int DT, bool SWAP>
int uneven_impl(const void* x, void* X, const int32_t* log2n, int64_t count, int seg_log2,
                int nthr) {
  using E = typename qftk::Store<DT>::T;
  int mx = 3;
  for (int64_t i = 0; i < count; ++i) mx = mx > log2n[i] ? mx : log2n[i];
  std::vector<float> sec = secants(mx);
  std::vector<int64_t> off, perm, large;
  std::vector<qftk::TileDesc> tiles;
  qftk::build_uneven_worklist(log2n, count, 10, off, tiles, perm, large);
  int races = 0;
  for (const auto& d : tiles) {
    const int r =
        tile_s_dispatch<DT, SWAP>(x, X, d.log2n, d.count, sec.data(), perm.data() + d.first);
    if (r < 0) return r;
    races += r;
  }
  // as the library runs them: 2^11 .. 2^14 one tile each, 2^15 and 2^16 the
  // two-pass path (2^12- and 2^13-cell segments), longer ones multi-pass
  for (int64_t i : large) {
    const int r =
        log2n[i] <= 14
            ? tile_s_dispatch<DT, SWAP>(x, X, log2n[i], 1, sec.data(), off.data() + i)
        : log2n[i] <= 16
            ? twopass_impl<DT, SWAP>((const E*)x + off[i], (E*)X + off[i], log2n[i] - 3, 1, 0)
            : multipass_impl<DT, SWAP>((const E*)x + off[i], (E*)X + off[i], log2n[i], 1,
                                       seg_log2, nthr, sec.data());
    if (r < 0) return r;
    races += r;
  }
  return races;
}

template <int DT, bool SWAP, int MC_LOG2>
int twopass_mc(const void* x, void* X, int64_t batch, int64_t grid) {
  using E = typename qftk::Store<DT>::T;
  constexpr int MC = 1 << MC_LOG2;
  // threads per workgroup: the GPU's (256 for 2^12-cell segments,
  // kTpBlock13 for 2^13), else <= 32
  constexpr int NT = MC_LOG2 == 13 ? qftk::kTpBlock13
                                   : MC_LOG2 >= 12 ? (2 * MC) / 32 : (MC < 32 ? MC : 32);
  constexpr int logn = MC_LOG2 + 3;
  const int64_t cells = batch << logn;
  std::vector<float> sec = secants(logn);
  std::vector<float2> heap(cells, make_float2(0.f, 0.f));
  int64_t races = 0;
  // pass A: both sides of one segment per workgroup, 4 workgroups per
  // transform, tracked writes of the heap buffer (no two workgroups may
  // write one cell)
  Tracker atr(NT);
  TPtr A{heap.data(), 0, &atr, cells};
  if (grid > 0) {
    // persistent launch: workgroup b takes tiles b, b + grid, .. with the
    // next tile's loads in flight during the current one (grid % 32 == 0)
    const int64_t ntiles = ((batch + 7) / 8) * 32;
    for (int64_t b = 0; b < grid; ++b) {
      const int64_t lc = 2 * MC + 1;
      std::vector<float2> lds(lc + (lc >> kEmuPad));
      Tracker ltr(NT);
      TPtr L{lds.data(), 0, &ltr, lc, kEmuPad};
      run_workgroup(NT, ltr, [&](int tid, auto sync, auto wsync) {
        tl_actor = b * NT + tid;
        qftk::tp_pass_a2_loop<DT, SWAP, MC_LOG2, NT, 64>((const E*)x, A, L, batch, ntiles, b,
                                                         grid, sec.data(), tid, sync, wsync);
      });
      if (ltr.oob) return -102;
      races += ltr.races;
    }
  }
  for (int64_t t = 0; t < batch && grid == 0; ++t) {
    for (int j = 0; j < 4; ++j) {
      const int64_t lc = 2 * MC + 1;
      std::vector<float2> lds(lc + (lc >> kEmuPad));
      Tracker ltr(NT);
      TPtr L{lds.data(), 0, &ltr, lc, kEmuPad};
      const E* xt = (const E*)x + (t << logn);
      run_workgroup(NT, ltr, [&](int tid, auto sync, auto wsync) {
        tl_actor = (t * 4 + j) * NT + tid;  // unique over all workgroups
        qftk::tp_pass_a2<DT, SWAP, MC_LOG2, NT, 64>(xt, A + (t << logn), L, j, sec.data(), tid,
                                                    sync, wsync);
      });
      if (ltr.oob) return -102;
      races += ltr.races;
    }
  }
  atr.end_phase();
  if (atr.oob) return -103;
  races += atr.races;
  // pass B: N/8 items per transform, tracked reads of the heap buffer
  Tracker gtr(1);
  TPtr G{heap.data(), 0, &gtr, cells};
  tl_slot = 0;
  for (int64_t t = 0; t < batch; ++t) {
    for (int k = 0; k < (1 << (logn - 3)); ++k) {
      set_item_actor(t * 100000 + k);
      qftk::tp_pass_b<DT, SWAP, MC_LOG2>(G + (t << logn), (E*)X + (t << logn), k);
    }
  }
  gtr.end_phase();
  if (gtr.oob) return -101;
  return (int)(races + gtr.races);
}

template <int DT, bool SWAP>
int twopass_impl(const void* x, void* X, int mc_log2, int64_t batch, int64_t grid) {
  switch (mc_log2) {
    case 3: return twopass_mc<DT, SWAP, 3>(x, X, batch, grid);
    case 4: return twopass_mc<DT, SWAP, 4>(x, X, batch, grid);
    case 5: return twopass_mc<DT, SWAP, 5>(x, X, batch, grid);
    case 7: return twopass_mc<DT, SWAP, 7>(x, X, batch, grid);
    case 10: return twopass_mc<DT, SWAP, 10>(x, X, batch, grid);
    case 12: return twopass_mc<DT, SWAP, 12>(x, X, batch, grid);
    case 13: return twopass_mc<DT, SWAP, 13>(x, X, batch, grid);
    default: return -5;
  }
}

}  // namespace

extern "C" {

// Two-pass path with segments of 2^mc_log2 cells (N = 8 * 2^mc_log2).
// grid = 0: one workgroup per tile of pass A; else a persistent grid of that
// many workgroups (a multiple of 32, as the library launches it).
int emu_twopass(int dt, int swap, const void* x, void* X, int mc_log2, int64_t batch,
                int64_t grid) {
  if (batch < 1 || grid < 0 || grid % 32 != 0) return -1;
  if (dt == 0) return swap ? twopass_impl<0, true>(x, X, mc_log2, batch, grid)
                           : twopass_impl<0, false>(x, X, mc_log2, batch, grid);
  return swap ? twopass_impl<1, true>(x, X, mc_log2, batch, grid)
              : twopass_impl<1, false>(x, X, mc_log2, batch, grid);
}


// One workgroup of the specialised GPU tile kernel (Tact transforms): a
// contiguous batch, or, with offs != NULL, transforms at element offsets
// offs[0 .. Tact) (the persistent kernel of uneven plans).
int emu_tile_s(int dt, int swap, const void* x, void* X, int logn, int Tact,
               const int64_t* offs) {
  std::vector<float> sec = secants(logn < 3 ? 3 : logn);
  if (dt == 0) return swap ? tile_s_dispatch<0, true>(x, X, logn, Tact, sec.data(), offs)
                           : tile_s_dispatch<0, false>(x, X, logn, Tact, sec.data(), offs);
  return swap ? tile_s_dispatch<1, true>(x, X, logn, Tact, sec.data(), offs)
              : tile_s_dispatch<1, false>(x, X, logn, Tact, sec.data(), offs);
}

// The resident-grid kernel of an uneven group of 2^13- or 2^14-point
// transforms, one per tile (tiles: int4 per tile, (log2n, first, 1, 0)).
int emu_tile_pg(int dt, int swap, const void* x, void* X, int logn, const int32_t* tiles,
                const int64_t* offs, int64_t ntiles, int64_t grid) {
  if (ntiles < 1 || grid < 1 || (logn != 13 && logn != 14)) return -1;
  std::vector<float> sec = secants(logn);
  const int4* t = reinterpret_cast<const int4*>(tiles);
  if (dt != 0) return -1;
  if (logn == 13)
    return swap ? tile_pg_impl<0, true, 13>(x, X, t, offs, ntiles, grid, sec.data())
                : tile_pg_impl<0, false, 13>(x, X, t, offs, ntiles, grid, sec.data());
  return swap ? tile_pg_impl<0, true, 14>(x, X, t, offs, ntiles, grid, sec.data())
              : tile_pg_impl<0, false, 14>(x, X, t, offs, ntiles, grid, sec.data());
}

// The resident-grid tile kernel (tile_kernel_p) with `grid` workgroups.
int emu_tile_p(int dt, int swap, const void* x, void* X, int logn, int64_t batch,
               int64_t grid) {
  if (batch < 1 || grid < 1) return -1;
  std::vector<float> sec = secants(logn < 3 ? 3 : logn);
  if (dt == 0) return swap ? tile_p_dispatch<0, true>(x, X, logn, batch, grid, sec.data())
                           : tile_p_dispatch<0, false>(x, X, logn, batch, grid, sec.data());
  return swap ? tile_p_dispatch<1, true>(x, X, logn, batch, grid, sec.data())
              : tile_p_dispatch<1, false>(x, X, logn, batch, grid, sec.data());
}

// One workgroup of the real-input tile kernel (kind 0: rdft in0 -> out0;
// kind 1: DCT-0 in0 -> out0 and DST-0 in1 -> out1, either pair may be null).
int emu_tile_real(int kind, int dt, int logn, int64_t rows, const void* in0, const void* in1,
                  void* out0, void* out1) {
  std::vector<float> sec = secants(logn < 3 ? 3 : logn);
  if (dt == 0) return kind == 0 ? tile_real_dispatch<0, 0>(logn, rows, in0, in1, out0, out1, sec.data())
                                : tile_real_dispatch<0, 1>(logn, rows, in0, in1, out0, out1, sec.data());
  return kind == 0 ? tile_real_dispatch<1, 0>(logn, rows, in0, in1, out0, out1, sec.data())
                   : tile_real_dispatch<1, 1>(logn, rows, in0, in1, out0, out1, sec.data());
}

// Multi-pass path of a real-input plan with 2^seg_log2-cell segments.
int emu_multipass_real(int kind, int dt, int logn, int64_t rows, const void* in0,
                       const void* in1, void* out0, void* out1, int seg_log2, int nthr) {
  if (logn < 4 || logn > 24 || rows < 1 || nthr < 1) return -1;
  std::vector<float> sec = secants(logn);
  return dt == 0 ? multipass_real_impl<0>(kind, logn, rows, in0, in1, out0, out1, seg_log2, nthr,
                                          sec.data())
                 : multipass_real_impl<1>(kind, logn, rows, in0, in1, out0, out1, seg_log2, nthr,
                                          sec.data());
}

int emu_multipass(int dt, int swap, const void* x, void* X, int logn, int64_t batch,
                  int seg_log2, int nthr) {
  if (logn < 4 || logn > 24 || batch < 1 || nthr < 1) return -1;
  std::vector<float> sec = secants(logn);
  if (dt == 0)
    return swap ? multipass_impl<0, true>(x, X, logn, batch, seg_log2, nthr, sec.data())
                : multipass_impl<0, false>(x, X, logn, batch, seg_log2, nthr, sec.data());
  return swap ? multipass_impl<1, true>(x, X, logn, batch, seg_log2, nthr, sec.data())
              : multipass_impl<1, false>(x, X, logn, batch, seg_log2, nthr, sec.data());
}

int emu_uneven(int dt, int swap, const void* x, void* X, const int32_t* log2n, int64_t count,
               int seg_log2, int nthr) {
  if (count < 1 || nthr < 1) return -1;
  if (dt == 0) return swap ? uneven_impl<0, true>(x, X, log2n, count, seg_log2, nthr)
                           : uneven_impl<0, false>(x, X, log2n, count, seg_log2, nthr);
  return swap ? uneven_impl<1, true>(x, X, log2n, count, seg_log2, nthr)
              : uneven_impl<1, false>(x, X, log2n, count, seg_log2, nthr);
}

// Checks the race model on a 128-thread workgroup (two wavefronts) over a
// 128-cell buffer: every thread writes cell tid, then, after `order` (0:
// nothing, 1: a wave-level sync, 2: a workgroup barrier), reads cell
// partner(tid) = tid ^ 1 (its own wavefront) for same_wave != 0, else
// (tid + 64) % 128 (the other wavefront).  Returns the races found.
int emu_race_model_check(int order, int same_wave) {
  constexpr int nthr = 128;
  std::vector<float2> buf(nthr);
  Tracker tr(nthr);
  TPtr B{buf.data(), 0, &tr, nthr};
  run_workgroup(nthr, tr, [&](int tid, auto sync, auto wsync) {
    B[tid] = make_float2((float)tid, 0.f);
    if (order == 1) wsync();
    if (order == 2) sync();
    const int p = same_wave ? (tid ^ 1) : (tid + 64) % nthr;
    const float2 v = B[p];
    (void)v;
  });
  return (int)tr.races;
}

// The fixed-point transform (qft_fixed.hpp) of `batch` complex int32
// signals of 2^logn points, x, X as int32 pairs, one emulated workgroup of
// nthr threads per transform with tracked heap buffers, input and output.
// Returns the races found, or a negative code.
int emu_fixed(const int32_t* x, int32_t* X, int logn, int64_t batch, int nthr, int fuse2) {
  if (logn < 1 || logn > 16 || batch < 1 || nthr < 1) return -1;
  const int64_t N = (int64_t)1 << logn;
  std::vector<int> H((size_t)std::max<int64_t>(N / 4, 2)), shift(32);
  qftk::fx::fill_table_q(H.data(), shift.data(), logn);
  const qftk::fx::Table tab{H.data(), shift.data()};
  int64_t races = 0;
  for (int64_t b = 0; b < batch; ++b) {
    std::vector<int2> b0((size_t)N), b1((size_t)N);
    Tracker tr(nthr);
    IPtr B0{b0.data(), 0, &tr, N}, B1{b1.data(), 0, &tr, N};
    IPtr xi{(int2*)(const_cast<int32_t*>(x)) + b * N, 0, &tr, N};
    IPtr Xo{(int2*)X + b * N, 0, &tr, N};
    // at most one wavefront of threads: ordered by wavefront syncs alone, as
    // on the GPU
    run_workgroup(nthr, tr, [&](int tid, auto sync, auto wsync) {
      if (nthr <= 64)
        qftk::fx::transform(xi, Xo, B0, B1, logn, tab, tid, nthr, wsync, fuse2 != 0);
      else
        qftk::fx::transform(xi, Xo, B0, B1, logn, tab, tid, nthr, sync, fuse2 != 0);
    });
    if (tr.oob) return -100;
    races += tr.races;
  }
  return (int)races;
}

// The library's integer constant table (host code of qft_fixed.hpp).
int emu_fixed_table(int log2n, int32_t* H, int32_t* shift) {
  if (log2n < 1 || log2n > 24) return -1;
  qftk::fx::fill_table_q(H, shift, log2n);
  return 0;
}

// Multi-pass path with a given split of the global passes (most forward
// rounds, backward rounds, chain levels per pass).
int emu_multipass_levels(int swap, const void* x, void* X, int logn, int64_t batch, int seg_log2,
                         int nthr, int fwd, int bwd, int chain) {
  if (logn < 4 || logn > 24 || batch < 1 || nthr < 1) return -1;
  if (fwd < 1 || fwd > 5 || bwd < 1 || bwd > 5 || chain < 1 || chain > 5) return -1;
  std::vector<float> sec = secants(logn);
  const qftk::MpLevels lv{fwd, bwd, chain};
  return swap ? multipass_impl<0, true>(x, X, logn, batch, seg_log2, nthr, sec.data(), lv)
              : multipass_impl<0, false>(x, X, logn, batch, seg_log2, nthr, sec.data(), lv);
}

// The library's schedule cache (host code shared with libqft.so).
int emu_cache_store(const char* path, const char* key, const char* name) {
  return qftk::schedule_cache_store(path, key, name) ? 1 : 0;
}

// 1 and the name in out[0 .. cap) if the key is found, else 0.
int emu_cache_lookup(const char* path, const char* key, char* out, int cap) {
  std::string name;
  if (!qftk::schedule_cache_lookup(path, key, name) || cap < 1) return 0;
  std::strncpy(out, name.c_str(), (size_t)cap - 1);
  out[cap - 1] = '\0';
  return 1;
}

// The cache path the library would use (environment read now).
int emu_cache_path(char* out, int cap) {
  const std::string p = qftk::schedule_cache_path();
  if (cap < 1) return -1;
  std::strncpy(out, p.c_str(), (size_t)cap - 1);
  out[cap - 1] = '\0';
  return (int)p.size();
}

}  // extern "C"
