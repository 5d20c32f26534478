// Device building blocks of the improved-QFT transform for gfx950.
//
// Work layout ("heap layout") of one transform of length N in a buffer W of N
// complex FP32 cells, after the real/imaginary split and real fold
// (Pasquini Sec. 4.1-4.2).  Both real signals of a complex transform follow
// the same control flow, so each cell holds the pair (value from Re x, value
// from Im x) as one float2 and every step below is a real-coefficient linear
// map applied to both components.
//
//   cells [0, N/2)   DCT side:  c(n) = x(n) + x(N-n), the s_dc_tt signal
//   cells [N/2, N)   DST side:  d(n) = x(n) - x(N-n), the s_ds_tt signal
//
// The repeated even/odd time split of ``dct``/``dst`` (Sec. 5.2.1, Sec. 3.1
// and the even-time halving of Sec. 3.4) peels from c the odd-time signals
// s_dc_ot of periodizations N, N/2, ...: the one of periodization P holds
// c(n) for n = (N/P)(2m+1), m < P/4, and is a DCT-II of length M = P/4.
// It is stored at cells [M, 2M) of the DCT side, position m.  Cell 0 holds
// c(0); cell N/2 (the first DST-side cell, which the DST side never uses)
// holds c(N/2).  The DST side is the same with DST-II blocks, d(N/4) (the
// ``dst`` base case) at cell N/2 + 1.  So every block of size M >= 1 sits at
// [M, 2M) and, for any S, the cells [S, N/2) of a side split into aligned
// segments [jS, (j+1)S), j >= 1, that cover exactly the blocks of size >= S.
//
// Forward sweep (time domain, Sec. 5.2.2-5.2.3): for S = N/4, N/8, .., 2 every
// aligned segment y of size S with j >= 1 is folded,
//     u(p) = y(p) + y(S-1-p),  v(p) = y(p) - y(S-1-p),  p < S/2,
// the harmonic separation of eqs. qft_1/qft_2.  DCT side: u goes to the first
// half (dct_ot of half size, even harmonics after the halving of Sec. 3.3) and
// v times the secant h_{S/2}(p) = 1/(2 cos(pi (2p+1)/(2S))) to the second
// half (dct_oo: eq. qft_38A then even-harmonic halving, i.e. again a dct_ot
// of half size).  DST side: the roles of u and v swap (Sec. 3.2, DST case).
//
// Backward sweep (frequency domain), S = 2, 4, .., N/4, segments j >= 1, the
// two halves A (first) and T (second) holding natural-order outputs:
//   DCT: Y(2i) = A(i), Y(2i+1) = T(i) + T(i+1), T(S/2) = 0
//        (interleave of eq. qft_4B; eq. qft_38C and the corrected eq. qft_38B)
//   DST (cell p holds harmonic p+1): Y(2i+1) = A(i), Y(2i) = T(i-1) + T(i),
//        T(-1) = 0 (the dst_oo special case at k = 1).
//
// Chain (``dct``/``dst`` backward, eqs. qft_5C, qft_5D, qft_6), P = 4 .. N:
//   DCT: D_P(k) = E(k) + O(k), D_P(P/2-k) = E(k) - O(k) (k < P/4),
//        D_P(P/4) = E(P/4), with E = D_{P/2} at cells [0, P/4) plus cell N/2
//        for E(P/4), O the DCT-II block at [P/4, P/2); D_P(k) -> cell k,
//        D_P(P/2) -> cell N/2.  Base P = 2: (c(0) + c(N/2), c(0) - c(N/2)).
//   DST: S_P(k) = O(k) + E(k), S_P(P/2-k) = O(k) - E(k) (1 <= k < P/4),
//        S_P(P/4) = O(P/4); E(k) at cell k, O(k) at cell P/4 + k - 1.
//        Base P = 4 (identity).
//
// Combine (cdft, Sec. 4.1): X(k) = C(k) - i S(k), X(N-k) = C(k) + i S(k)
// for 0 < k < N/2 with C(k) at DCT cell k and S(k) at DST cell k;
// X(0) = C(0), X(N/2) = C(N/2) (cell N/2).
//
// Every routine below is written for any pointer the compiler can resolve
// after inlining (LDS or global); loops are strided over the calling
// workgroup's threads (tid, nthr).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

// Every routine is __host__ __device__ so that the unchanged source can also
// be run on the CPU (tests drive it with emulated workgroups); barriers are a
// template functor (DevSync on the GPU).
#define QFT_HD __host__ __device__ __forceinline__

namespace qftk {

QFT_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
QFT_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
QFT_HD float2 cscale(float2 a, float h) { return make_float2(a.x * h, a.y * h); }

// ---------------------------------------------------------------------------
// Element I/O: FP32 or FP16 storage, optional re/im swap (adjoint = swap F swap)
// ---------------------------------------------------------------------------
template <int DT> struct Store;
template <> struct Store<0> {
  using T = float2;
  static QFT_HD float2 cvt(T v) { return v; }
  static QFT_HD float2 ld(const T* p, int64_t i) { return p[i]; }
  static QFT_HD void st(T* p, int64_t i, float2 v) { p[i] = v; }
};
template <> struct Store<1> {
  using T = __half2;
  static QFT_HD float2 cvt(T v) { return __half22float2(v); }
  static QFT_HD float2 ld(const T* p, int64_t i) { return __half22float2(p[i]); }
  static QFT_HD void st(T* p, int64_t i, float2 v) { p[i] = __float22half2_rn(v); }
};

// Real element storage (real-input entry points): FP32 or FP16.
template <int DT> struct RStore;
template <> struct RStore<0> {
  using T = float;
  static QFT_HD float ld(const T* p, int64_t i) { return p[i]; }
  static QFT_HD void st(T* p, int64_t i, float v) { p[i] = v; }
};
template <> struct RStore<1> {
  using T = __half;
  static QFT_HD float ld(const T* p, int64_t i) { return __half2float(p[i]); }
  static QFT_HD void st(T* p, int64_t i, float v) { p[i] = __float2half_rn(v); }
};

template <bool SWAP> QFT_HD float2 sw(float2 v) {
  if constexpr (SWAP) return make_float2(v.y, v.x);
  else return v;
}

// ---------------------------------------------------------------------------
// Forward rounds on one register group.  K consecutive rounds S, S/2, ..,
// S/2^(K-1) on segment j of one side.  With G = S >> K >= 2, the group of
// lane-offset x < G/2 is the closed cell set
//   { j S + c G + x, j S + c G + G-1-x : c < 2^K }
// (register e[2c] and e[2c+1]); each round maps it onto itself.  With G == 1
// (the last rounds, S = 2^K) the group is the whole segment.  With skip0 set
// (the side starts at heap cell 0), rounds whose segment is [0, S') of the
// side are not blocks and are skipped.
// ---------------------------------------------------------------------------
template <int K, bool DST, typename SP>
QFT_HD void fwd_group(SP sd, int S, int j, int x, const float* __restrict__ sec, bool skip0) {
  const int G = S >> K;
  const int base = j * S;
  constexpr int NE = 2 << K;
  float2 e[NE];
#pragma unroll
  for (int c = 0; c < (1 << K); ++c) {
    e[2 * c] = sd[base + c * G + x];
    e[2 * c + 1] = sd[base + c * G + G - 1 - x];
  }
#pragma unroll
  for (int m = K; m >= 1; --m) {
    const int span = 1 << m, half = span >> 1;
    const int L = G << (m - 1);  // S'/2, secant slice
    float2 o[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) o[i] = e[i];
#pragma unroll
    for (int c0 = 0; c0 < (1 << K); c0 += span) {
      if (skip0 && j == 0 && c0 == 0) continue;
#pragma unroll
      for (int cc = 0; cc < half; ++cc) {
        const int c = c0 + cc, cm = c0 + span - 1 - cc;
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          const float2 a = e[2 * c + f], b = e[2 * cm + 1 - f];
          const int u = cc * G + (f ? G - 1 - x : x);
          const float hsec = sec[L + u];
          const float2 s = cadd(a, b), d = csub(a, b);
          o[2 * c + f] = DST ? d : s;
          o[2 * (c + half) + f] = cscale(DST ? s : d, hsec);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) e[i] = o[i];
  }
#pragma unroll
  for (int c = 0; c < (1 << K); ++c) {
    sd[base + c * G + x] = e[2 * c];
    sd[base + c * G + G - 1 - x] = e[2 * c + 1];
  }
}

// ---------------------------------------------------------------------------
// Chain groups (closed, in place).  DCT side pointer dc (cells [0, n/2)),
// cell n/2 passed as `top` (pointer to the cell holding E(P/4)/D_P(P/2)).
// g = 0: the k = 0 triple; 1 <= g <= P/8: the pair (g, P/4 - g)
// (self-paired at g = P/8).
// ---------------------------------------------------------------------------
template <typename SP>
QFT_HD void chain_dct_group(SP dc, SP top, int P, int g) {
  const int q = P >> 2;
  if (g == 0) {
    const float2 E0 = dc[0], O0 = dc[q], Eq = *top;
    dc[0] = cadd(E0, O0);
    *top = csub(E0, O0);
    dc[q] = Eq;
    return;
  }
  const int k = g, kp = q - g;
  if (k == kp) {
    const float2 E = dc[k], O = dc[q + k];
    dc[k] = cadd(E, O);
    dc[q + k] = csub(E, O);  // cell P/2 - k = q + k when k = P/8
    return;
  }
  const float2 Ek = dc[k], Ok = dc[q + k], Ep = dc[kp], Op = dc[q + kp];
  dc[k] = cadd(Ek, Ok);
  dc[q + kp] = csub(Ek, Ok);  // P/2 - k
  dc[kp] = cadd(Ep, Op);
  dc[q + k] = csub(Ep, Op);   // P/2 - kp
}

// DST side pointer ds (cell p of the side).  g = 0: the triple
// {1, P/4, P/2-1}; 1 <= g <= P/8 - 1: the pair k = g+1, k' = P/4 + 1 - k.
template <typename SP>
QFT_HD void chain_dst_group(SP ds, int P, int g) {
  const int q = P >> 2;
  if (g == 0) {
    const float2 E1 = ds[1], O1 = ds[q], Oq = ds[2 * q - 1];
    ds[1] = cadd(O1, E1);
    ds[2 * q - 1] = csub(O1, E1);
    ds[q] = Oq;
    return;
  }
  const int k = g + 1, kp = q + 1 - k;
  const float2 Ek = ds[k], Ok = ds[q + k - 1], Ep = ds[kp], Op = ds[q + kp - 1];
  ds[k] = cadd(Ok, Ek);
  ds[q + kp - 1] = csub(Ok, Ek);  // P/2 - k
  ds[kp] = cadd(Op, Ep);
  ds[q + k - 1] = csub(Op, Ep);   // P/2 - kp
}


// ---------------------------------------------------------------------------
// LDS pointer with padding: logical cell c is stored at base[c + (c >> PS)],
// one spare cell per 2^PS cells, so that threads owning runs of cells at a
// power-of-two stride do not collide on LDS banks.  PS >= 16 means no padding.
// ---------------------------------------------------------------------------
template <int PS>
struct PadPtr {
  float2* base;
  int off;
  QFT_HD float2& operator[](int i) const {
    const int c = off + i;
    return base[PS >= 16 ? c : c + (c >> (PS & 15))];
  }
  QFT_HD float2& operator*() const { return (*this)[0]; }
  QFT_HD PadPtr operator+(int d) const { return PadPtr{base, off + d}; }
};

template <int PS>
QFT_HD constexpr int padded_cells(int cells) {
  return PS >= 16 ? cells : cells + (cells >> PS);
}

// Row of a buffer at cell a, with the address arithmetic of the padding done
// once: r[k] is cell a + k for k a multiple of 2^PS (the padding inside
// [a, a + k) is k >> PS cells wherever a lies), r.run(e) is cell a + e for
// the cells of a's own 2^PS-cell block (no padding in between).  Buffers
// without padding (global memory) get the plain offset pointer.
template <int PS>
struct PadRow {
  float2* p;
  QFT_HD float2& operator[](int k) const { return p[PS >= 16 ? k : k + (k >> (PS & 15))]; }
  QFT_HD float2& run(int e) const { return p[e]; }
};

// Callers index rows with multiples of kRowCells cells (the padding block
// must divide it) and anchor them at cells >= 0 of the buffer.
constexpr int kRowCells = 16;

template <int PS>
QFT_HD PadRow<PS> pad_row(const PadPtr<PS>& sd, int a) {
  static_assert(PS >= 16 || (1 << PS) <= kRowCells, "row offsets are whole padding blocks");
  const int c = sd.off + a;
  return PadRow<PS>{sd.base + (PS >= 16 ? c : c + (c >> (PS & 15)))};
}

template <typename SP>
struct PlainRow {
  SP p;
  QFT_HD decltype(auto) operator[](int k) const { return p[k]; }
  QFT_HD decltype(auto) run(int e) const { return p[e]; }
};

template <typename SP>
QFT_HD PlainRow<SP> pad_row(const SP& sd, int a) {
  return PlainRow<SP>{sd + a};
}

// ---------------------------------------------------------------------------
// Fused innermost rounds: forward rounds S = 2^K .. 2 and then backward
// rounds S = 2 .. 2^K on the whole segment j of 2^K cells, in registers.
// ---------------------------------------------------------------------------
template <int K, bool DST, typename SP>
QFT_HD void tail_group(SP sd, int j, const float* __restrict__ sec, bool skip0) {
  constexpr int S = 1 << K;
  const int base = j * S;
  float2 e[S];
#pragma unroll
  for (int c = 0; c < S; ++c) e[c] = sd[base + c];
#pragma unroll
  for (int m = K; m >= 1; --m) {
    const int span = 1 << m, half = span >> 1;
#pragma unroll
    for (int c0 = 0; c0 < S; c0 += span) {
      if (skip0 && j == 0 && c0 == 0) continue;
#pragma unroll
      for (int cc = 0; cc < half / 2 + (half & 1); ++cc) {
        // butterflies cc and half-1-cc touch cells {cc, span-1-cc} and
        // {half-1-cc, half+cc}; outputs go to {cc, half+cc, half-1-cc, span-1-cc}
        const int c2 = half - 1 - cc;
        const float2 a1 = e[c0 + cc], b1 = e[c0 + span - 1 - cc];
        const float2 a2 = e[c0 + c2], b2 = e[c0 + span - 1 - c2];
        const float h1 = sec[half + cc], h2 = sec[half + c2];
        const float2 s1 = cadd(a1, b1), d1 = csub(a1, b1);
        const float2 s2 = cadd(a2, b2), d2 = csub(a2, b2);
        e[c0 + cc] = DST ? d1 : s1;
        e[c0 + half + cc] = cscale(DST ? s1 : d1, h1);
        if (c2 != cc) {
          e[c0 + c2] = DST ? d2 : s2;
          e[c0 + half + c2] = cscale(DST ? s2 : d2, h2);
        }
      }
    }
  }
#pragma unroll
  for (int m = 1; m <= K; ++m) {
    const int span = 1 << m, half = span >> 1;
#pragma unroll
    for (int c0 = 0; c0 < S; c0 += span) {
      if (skip0 && j == 0 && c0 == 0) continue;
      float2 y[S];
#pragma unroll
      for (int i = 0; i < half; ++i) {
        const float2 A = e[c0 + i], T = e[c0 + half + i];
        if (!DST) {
          y[2 * i] = A;
          y[2 * i + 1] = (i + 1 < half) ? cadd(T, e[c0 + half + i + 1]) : T;
        } else {
          y[2 * i + 1] = A;
          y[2 * i] = (i >= 1) ? cadd(e[c0 + half + i - 1], T) : T;
        }
      }
#pragma unroll
      for (int i = 0; i < span; ++i) e[c0 + i] = y[i];
    }
  }
#pragma unroll
  for (int c = 0; c < S; ++c) sd[base + c] = e[c];
}

// ---------------------------------------------------------------------------
// K backward rounds S/2^(K-1) .. S on segment j (input: its 2^K sub-segments
// of G = S/2^K cells, each a natural-order DCT-II/DST-II of length G).  The
// thread with lane offset i < G computes the natural-order outputs
// i*2^K .. i*2^K + 2^K - 1 of the segment.  Level by level, sub-segment pairs
// (A, T) become Y(2e) = A(e), Y(2e+1) = T(e) + T(e+1) (DCT) or
// Y(2e+1) = A(e), Y(2e) = T(e-1) + T(e) (DST); the one neighbour beyond the
// thread's block is always an A-chain pass-through of an input cell at i+1
// (DCT) or i-1 (DST), so it is loaded, not recomputed: 2^(K+1) - 1 loads,
// K 2^(K-1) additions, no redundant arithmetic.
// ---------------------------------------------------------------------------
template <int K, bool DST>
QFT_HD void bwd_group_levels(float2 (&cur)[1 << K], float2 (&halo)[1 << K], float2 (&y)[1 << K]) {
  constexpr int R = 1 << K;
#pragma unroll
  for (int m = 1; m <= K; ++m) {
    const int len = 1 << m, hl = len >> 1;  // values per segment at level m / m-1
    float2 nxt[R], nh[R];
#pragma unroll
    for (int c = 0; c < (R >> m); ++c) {
      const int a0 = (2 * c) * hl, t0 = (2 * c + 1) * hl;  // A and T in cur
#pragma unroll
      for (int e = 0; e < hl; ++e) {
        const float2 A = cur[a0 + e], T = cur[t0 + e];
        if (!DST) {
          nxt[c * len + 2 * e] = A;
          nxt[c * len + 2 * e + 1] = cadd(T, (e + 1 < hl) ? cur[t0 + e + 1] : halo[2 * c + 1]);
        } else {
          nxt[c * len + 2 * e + 1] = A;
          nxt[c * len + 2 * e] = cadd((e >= 1) ? cur[t0 + e - 1] : halo[2 * c + 1], T);
        }
      }
      nh[c] = halo[2 * c];
    }
#pragma unroll
    for (int c = 0; c < R; ++c) cur[c] = nxt[c];
#pragma unroll
    for (int c = 0; c < (R >> m); ++c) halo[c] = nh[c];
  }
#pragma unroll
  for (int c = 0; c < R; ++c) y[c] = cur[c];
}

template <int K, bool DST, typename SP>
QFT_HD void bwd_group_load(SP sd, int S, int j, int i, float2 (&y)[1 << K]) {
  constexpr int R = 1 << K;
  const int G = S >> K;
  const int base = j * S;
  float2 cur[R], halo[R];
#pragma unroll
  for (int c = 0; c < R; ++c) cur[c] = sd[base + c * G + i];
  const bool has = DST ? (i >= 1) : (i + 1 < G);
  const int hi = DST ? i - 1 : i + 1;
#pragma unroll
  for (int c = 0; c < R; ++c)
    halo[c] = (c > 0 && has) ? (float2)sd[base + c * G + hi] : make_float2(0.f, 0.f);
  bwd_group_levels<K, DST>(cur, halo, y);
}

// bwd_group_load with the sub-segment length G known at compile time and the
// segment starting at cell base: row accesses when G is a multiple of
// kRowCells.
template <int K, int G, bool DST, typename SP>
QFT_HD void bwd_group_load_s(SP sd, int base, int i, float2 (&y)[1 << K]) {
  constexpr int R = 1 << K;
  float2 cur[R], halo[R];
  const bool has = DST ? (i >= 1) : (i + 1 < G);
  const int hi = has ? (DST ? i - 1 : i + 1) : i;
  if constexpr (G % kRowCells == 0) {
    const auto rc = pad_row(sd, base + i);
    const auto rh = pad_row(sd, base + hi);
#pragma unroll
    for (int c = 0; c < R; ++c) cur[c] = rc[c * G];
#pragma unroll
    for (int c = 0; c < R; ++c)
      halo[c] = (c > 0 && has) ? (float2)rh[c * G] : make_float2(0.f, 0.f);
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) cur[c] = sd[base + c * G + i];
#pragma unroll
    for (int c = 0; c < R; ++c)
      halo[c] = (c > 0 && has) ? (float2)sd[base + c * G + hi] : make_float2(0.f, 0.f);
  }
  bwd_group_levels<K, DST>(cur, halo, y);
}

// The segment j == 0 of a side head (heap) holds the blocks M = 2G, 4G, ..,
// S/2 that still need a rounds each (M = G 2^a); the lane-i thread loads the
// a-level groups of all of them into out[] (2^K - 2 values).
template <int K, bool DST, int A, typename SP>
QFT_HD void bwd_head_load(SP sd, int G, int i, float2* out) {
  if constexpr (A < K) {
    float2 y[1 << A];
    bwd_group_load<A, DST>(sd, G << A, 1, i, y);
#pragma unroll
    for (int e = 0; e < (1 << A); ++e) out[e] = y[e];
    bwd_head_load<K, DST, A + 1>(sd, G, i, out + (1 << A));
  }
}

template <int K, int A, typename SP>
QFT_HD void bwd_head_store(SP sd, int G, int i, const float2* in) {
  if constexpr (A < K) {
    const int M = G << A;
#pragma unroll
    for (int e = 0; e < (1 << A); ++e) sd[M + i * (1 << A) + e] = in[e];
    bwd_head_store<K, A + 1>(sd, G, i, in + (1 << A));
  }
}

// bwd_head_load / bwd_head_store with G known at compile time (row accesses;
// the outputs of one item are a run inside one padding block).
template <int K, bool DST, int A, int G, typename SP>
QFT_HD void bwd_head_load_s(SP sd, int i, float2* out) {
  if constexpr (A < K) {
    float2 y[1 << A];
    bwd_group_load_s<A, G, DST>(sd, G << A, i, y);
#pragma unroll
    for (int e = 0; e < (1 << A); ++e) out[e] = y[e];
    bwd_head_load_s<K, DST, A + 1, G>(sd, i, out + (1 << A));
  }
}

template <int K, int A, int G, typename SP>
QFT_HD void bwd_head_store_s(SP sd, int i, const float2* in) {
  if constexpr (A < K) {
    const auto r = pad_row(sd, (G << A) + i * (1 << A));
#pragma unroll
    for (int e = 0; e < (1 << A); ++e) r.run(e) = in[e];
    bwd_head_store_s<K, A + 1, G>(sd, i, in + (1 << A));
  }
}

// ===========================================================================
// Sides.  A "side" is one half of a transform's heap (DCT or DST); the sides
// of a tile alternate DCT/DST, an isolated segment of a larger transform is
// a single side of fixed flavour.
// ===========================================================================
enum SideMode { SIDES_ALT = 0, SIDES_DCT = 1, SIDES_DST = 2 };

// DCT-0 / DST-0 chain level P = 2^p (p >= 1) for transform heap dc (length
// 2^logn): group g of the level (see chain_*_group).  Groups per transform:
// P = 2: 1; P = 4: 1; P >= 8: (1 + P/8) DCT + P/8 DST.
QFT_HD int chain_groups(int p) {
  return p <= 2 ? 1 : 1 + 2 * (1 << (p - 3));
}

template <typename WP>
QFT_HD void chain_item(WP dc, int logn, int p, int g) {
  const int h = 1 << (logn - 1);
  const int P = 1 << p;
  if (P == 2) {
    const float2 a = dc[0], b = dc[h];
    dc[0] = cadd(a, b);
    dc[h] = csub(a, b);
    return;
  }
  const int ngd = (P == 4) ? 1 : 1 + (P >> 3);
  if (g < ngd) chain_dct_group(dc, dc + h, P, g);
  else chain_dst_group(dc + h, P, g - ngd);
}

// ===========================================================================
// Multi-pass path (one transform too large for a workgroup).  Work items of
// the global passes over heap buffers of `batch` transforms (transform t at
// cell t 2^logn, DCT side first, DST side at + N/2).
// ===========================================================================
// Fold item i < batch * N/2 through an IO accessor (fetch + fold as in the
// tile body), transform slot t = i / (N/2).
template <class IO, typename WP>
QFT_HD void mp_fold_io_item(const IO& io, WP W, int logn, int64_t i) {
  const int n = 1 << logn, h = n >> 1;
  const int64_t t = i >> (logn - 1);
  const int m = (int)(i & (h - 1));
  auto w = W + (t << logn);
  typename IO::Raw r;
  io.fetch((int)t, m, r);
  float2 lo, hi;
  io.fold(r, m, lo, hi);
  if (m == 0) {
    w[0] = lo;
    w[h] = hi;
  } else {
    const int l = __builtin_ctz(m);
    const int cell = (n >> (l + 2)) + (m >> (l + 1));
    w[cell] = lo;
    w[h + cell] = hi;
  }
}

// forward group item i < 2*batch * 2^(logn-K-2): K rounds ending at
// S = 2^(hi-K+1) >= 4, in place (groups are closed cell sets).
template <int K, typename WP>
QFT_HD void mp_fwd_item(WP W, int logn, int hi, const float* sec, int64_t i) {
  const int lgside = logn - 1;
  const int lgGroups = lgside - K - 1;
  const int lgHalfG = hi - K - 1;
  const int64_t s = i >> lgGroups;
  const int g = (int)(i & ((1 << lgGroups) - 1));
  const int j = g >> lgHalfG;
  const int x = g & ((1 << lgHalfG) - 1);
  auto sd = W + (s << lgside);
  if (s & 1) fwd_group<K, true>(sd, 1 << hi, j, x, sec, true);
  else fwd_group<K, false>(sd, 1 << hi, j, x, sec, true);
}

// K backward rounds S = 2^(s-K+1) .. 2^s on every side, Win -> Wout; item
// i < 2*batch * 2^(logn-1-K).  With G = 2^(s-K), item (side, j, ii) of a
// segment j >= 1 of S cells computes outputs ii 2^K .. ii 2^K + 2^K - 1 of
// the segment (bwd_group_load).  The items of segment 0 take the side head:
// cell ii of [0, G) unchanged (cell 0 of the DST side is the chain's top
// cell) and the blocks M = G 2^a, a < K, which are complete after a more
// rounds, 2^K outputs per item in both cases.
template <int K, typename RP, typename WP>
QFT_HD void mp_bwd_group_item(RP Win, WP Wout, int logn, int s, int64_t i) {
  const int lgside = logn - 1;
  const int lgItems = lgside - K;
  const int lgG = s - K;
  const int64_t si = i >> lgItems;
  const int item = (int)(i & ((1 << lgItems) - 1));
  const int j = item >> lgG;
  const int ii = item & ((1 << lgG) - 1);
  auto sin = Win + (si << lgside);
  auto sout = Wout + (si << lgside);
  if (j > 0) {
    float2 y[1 << K];
    if (si & 1) bwd_group_load<K, true>(sin, 1 << s, j, ii, y);
    else bwd_group_load<K, false>(sin, 1 << s, j, ii, y);
    const int o = (j << s) + (ii << K);
#pragma unroll
    for (int e = 0; e < (1 << K); ++e) sout[o + e] = y[e];
  } else {
    float2 hv[(1 << K) - 1];
    const float2 c = sin[ii];
    if (si & 1) bwd_head_load<K, true, 0>(sin, 1 << lgG, ii, hv);
    else bwd_head_load<K, false, 0>(sin, 1 << lgG, ii, hv);
    sout[ii] = c;
    bwd_head_store<K, 0>(sout, 1 << lgG, ii, hv);
  }
}



// The same backward rounds for the items of one wavefront of LANES lanes
// (lane = i mod LANES).  An item of a segment j >= 1 computes 2^K
// consecutive outputs, so storing them straight from each lane would spread
// every store instruction over LANES runs.  A segment holds 2^(hi-K) >=
// LANES items, so the wave's items belong to one segment of one side and
// their outputs are LANES * 2^K consecutive cells: the wave passes them
// through its LDS rows ws (LANES * ROW cells) in chunks of CH outputs per
// lane (a 128-byte line per lane for CH = 16) and stores each chunk with
// unit-stride lanes.  Items of segment 0 (the side head, whole waves of it)
// store directly.  Needs hi - K >= log2 LANES.
template <int K>
struct MpBwdStage {
  static constexpr int R = 1 << K;
  static constexpr int CH = R < 16 ? R : 16;
  static constexpr int ROW = CH + 1;  // padded row of one lane's chunk
};

template <int K, int LANES, typename RP, typename WP, typename SP, class WSync>
QFT_HD void mp_bwd_wave_item(RP Win, WP Wout, SP ws, int logn, int hi, int64_t i, int lane,
                             WSync wsync) {
  using St = MpBwdStage<K>;
  constexpr int R = St::R, CH = St::CH, ROW = St::ROW;
  const int lgside = logn - 1;
  const int lgItems = lgside - K;
  const int lgG = hi - K;
  const int64_t si = i >> lgItems;
  const int item = (int)(i & ((1 << lgItems) - 1));
  const int j = item >> lgG;
  if (j == 0) {  // uniform over the wave
    mp_bwd_group_item<K>(Win, Wout, logn, hi, i);
    return;
  }
  const int ii = item & ((1 << lgG) - 1);
  float2 y[R];
  if (si & 1) bwd_group_load<K, true>(Win + (si << lgside), 1 << hi, j, ii, y);
  else bwd_group_load<K, false>(Win + (si << lgside), 1 << hi, j, ii, y);
  // lane 0's outputs start here, lane l's at + l * R
  auto out = Wout + (si << lgside) + ((int64_t)j << hi) + ((int64_t)(ii - lane) << K);
#pragma unroll
  for (int c = 0; c < R / CH; ++c) {
#pragma unroll
    for (int e = 0; e < CH; ++e) ws[lane * ROW + e] = y[c * CH + e];
    wsync();
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      const int f = r * LANES + lane;  // cell f of the chunk: lane f / CH, output f % CH
      out[(f / CH) * R + c * CH + (f % CH)] = (float2)ws[(f / CH) * ROW + (f % CH)];
    }
    wsync();
  }
}

// ===========================================================================
// Compile-time specialised sweeps.  Sizes, round schedule and the thread ->
// group mapping are template parameters, so that index arithmetic folds into
// LDS instruction offsets and no bounds guards remain.  NS = sides in the
// buffer (each 2^LGS cells, side s at W + s*2^LGS), NT = threads, MODE as in
// SideMode (SIDES_ALT: even sides DCT, odd sides DST).
// ===========================================================================
template <int A, int B> struct cmin { static constexpr int v = A < B ? A : B; };

// Thread -> item map of one LDS pass over NS sides of 2^LGS cells, in items
// of 2^LGE consecutive (tail, backward) or segment-spanning (forward) cells,
// for NT threads in waves of WAVE lanes.  Where every thread gets the same
// number of items, wave w takes items [w I, (w+1) I), I = items per wave, in
// lane-consecutive order: it then touches only the cells [w C, (w+1) C) of
// the buffer (C = cells per wave) whenever the pass's segments (2^LGSEG
// cells) are no longer than C.  Two such passes in a row need no workgroup
// barrier between them, only the wave's own ordering.
template <int NS, int LGS, int NT, int WAVE, int LGE, int LGSEG>
struct PassMap {
  static constexpr int total = NS << (LGS - LGE);
  static constexpr int NI = (total + NT - 1) / NT;
  static constexpr int WE = NT < WAVE ? NT : WAVE;
  static constexpr int NW = NT / WE;
  static_assert(NW == 1 || NT % WAVE == 0, "whole waves");
  static constexpr bool blocked = NW > 1 && total == NI * NT;
  static constexpr int C = blocked ? NI * WE << LGE : 0;
  static constexpr bool local = NW == 1 || (blocked && (1 << LGSEG) <= C);
  static QFT_HD int item(int tid, int it) {
    if constexpr (blocked) {
      const int w = tid / WE;
      return w * (NI * WE) + it * WE + (tid - w * WE);
    } else {
      return tid + it * NT;
    }
  }
};

// The ordering between two LDS passes: the wave's own where both stay in
// the wave's cells, else a workgroup barrier.
template <bool WAVE_ONLY, class Sync, class WSync>
QFT_HD void pass_sync(Sync sync, WSync wsync) {
  if constexpr (WAVE_ONLY) wsync();
  else sync();
}

template <int K, int S, bool DST, typename SP>
QFT_HD void fwd_group_s(SP sd, int j, int x, const float* __restrict__ sec, bool skip0) {
  constexpr int G = S >> K;
  constexpr int NE = 2 << K;
  const int base = j * S;
  float2 e[NE];
  // rows at x and G-1-x when G is a multiple of kRowCells
  constexpr bool ROWS = G % kRowCells == 0;
  const auto rx = pad_row(sd, base + x);
  const auto rm = pad_row(sd, base + G - 1 - x);
#pragma unroll
  for (int c = 0; c < (1 << K); ++c) {
    if constexpr (ROWS) {
      e[2 * c] = rx[c * G];
      e[2 * c + 1] = rm[c * G];
    } else {
      e[2 * c] = sd[base + c * G + x];
      e[2 * c + 1] = sd[base + c * G + G - 1 - x];
    }
  }
#pragma unroll
  for (int m = K; m >= 1; --m) {
    const int span = 1 << m, half = span >> 1;
    const int L = G << (m - 1);
    float2 o[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) o[i] = e[i];
#pragma unroll
    for (int c0 = 0; c0 < (1 << K); c0 += span) {
      if (c0 == 0 && skip0 && j == 0) continue;
#pragma unroll
      for (int cc = 0; cc < half; ++cc) {
        const int c = c0 + cc, cm = c0 + span - 1 - cc;
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          const float2 a = e[2 * c + f], b = e[2 * cm + 1 - f];
          const float hsec = f ? sec[L + cc * G + G - 1 - x] : sec[L + cc * G + x];
          const float2 sm = cadd(a, b), df = csub(a, b);
          o[2 * c + f] = DST ? df : sm;
          o[2 * (c + half) + f] = cscale(DST ? sm : df, hsec);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) e[i] = o[i];
  }
#pragma unroll
  for (int c = 0; c < (1 << K); ++c) {
    if constexpr (ROWS) {
      rx[c * G] = e[2 * c];
      rm[c * G] = e[2 * c + 1];
    } else {
      sd[base + c * G + x] = e[2 * c];
      sd[base + c * G + G - 1 - x] = e[2 * c + 1];
    }
  }
}

// b with its sign bit flipped where mask has it set (mask 0: b itself).
QFT_HD float2 flip_sign(float2 b, unsigned mask) {
  return make_float2(__builtin_bit_cast(float, __builtin_bit_cast(unsigned, b.x) ^ mask),
                     __builtin_bit_cast(float, __builtin_bit_cast(unsigned, b.y) ^ mask));
}

// fwd_group_s for both sides in one code path: the DCT side keeps a + b and
// scales a - b, the DST side keeps a - b and scales a + b, so both are a + b'
// and (a - b') h with b' = b, or -b (exact) where dst_mask holds the sign bit.
template <int K, int S, typename SP>
QFT_HD void fwd_group_sf(SP sd, int j, int x, const float* __restrict__ sec, bool skip0,
                         unsigned dst_mask) {
  constexpr int G = S >> K;
  constexpr int NE = 2 << K;
  const int base = j * S;
  float2 e[NE];
  // rows at x and G-1-x when G is a multiple of kRowCells
  constexpr bool ROWS = G % kRowCells == 0;
  const auto rx = pad_row(sd, base + x);
  const auto rm = pad_row(sd, base + G - 1 - x);
#pragma unroll
  for (int c = 0; c < (1 << K); ++c) {
    if constexpr (ROWS) {
      e[2 * c] = rx[c * G];
      e[2 * c + 1] = rm[c * G];
    } else {
      e[2 * c] = sd[base + c * G + x];
      e[2 * c + 1] = sd[base + c * G + G - 1 - x];
    }
  }
#pragma unroll
  for (int m = K; m >= 1; --m) {
    const int span = 1 << m, half = span >> 1;
    const int L = G << (m - 1);
    float2 o[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) o[i] = e[i];
#pragma unroll
    for (int c0 = 0; c0 < (1 << K); c0 += span) {
      if (c0 == 0 && skip0 && j == 0) continue;
#pragma unroll
      for (int cc = 0; cc < half; ++cc) {
        const int c = c0 + cc, cm = c0 + span - 1 - cc;
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          const float2 a = e[2 * c + f], b = flip_sign(e[2 * cm + 1 - f], dst_mask);
          const float hsec = f ? sec[L + cc * G + G - 1 - x] : sec[L + cc * G + x];
          o[2 * c + f] = cadd(a, b);
          o[2 * (c + half) + f] = cscale(csub(a, b), hsec);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) e[i] = o[i];
  }
#pragma unroll
  for (int c = 0; c < (1 << K); ++c) {
    if constexpr (ROWS) {
      rx[c * G] = e[2 * c];
      rm[c * G] = e[2 * c + 1];
    } else {
      sd[base + c * G + x] = e[2 * c];
      sd[base + c * G + G - 1 - x] = e[2 * c + 1];
    }
  }
}

// SF: one branch-free code path for both sides (the side's sign mask at run
// time), else a branch per item between the two sides' own code.  Which is
// faster depends on the kernel (the branch-free one issues two more
// instructions per butterfly and no moves where the branches join).
template <int K, int HI, int LGS, int NS, int NT, int WAVE, int MODE, bool SKIP0, bool SF,
          typename WP>
QFT_HD void fwd_chunk_s(WP W, const float* sec, int tid) {
  using Map = PassMap<NS, LGS, NT, WAVE, K + 1, HI>;
  constexpr int lgGroups = LGS - K - 1;
  constexpr int total = Map::total;
  constexpr int NI = Map::NI;
  constexpr int lgHalfG = HI - K - 1;
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int i = Map::item(tid, it);
    if ((total % NT) != 0 && i >= total) break;
    const int s = i >> lgGroups;
    const int g = i & ((1 << lgGroups) - 1);
    const int j = g >> lgHalfG;
    const int x = g & ((1 << lgHalfG) - 1);
    auto sd = W + (s << LGS);
    const bool dst = MODE == SIDES_DST || (MODE == SIDES_ALT && (s & 1));
    if constexpr (SF) {
      fwd_group_sf<K, (1 << HI)>(sd, j, x, sec, SKIP0, dst ? 0x80000000u : 0u);
    } else {
      if (dst) fwd_group_s<K, (1 << HI), true>(sd, j, x, sec, SKIP0);
      else fwd_group_s<K, (1 << HI), false>(sd, j, x, sec, SKIP0);
    }
  }
}

template <int K, int LGS, int NS, int NT, int WAVE, int MODE, bool SKIP0, typename WP>
QFT_HD void tail_chunk_s(WP W, const float* sec, int tid) {
  using Map = PassMap<NS, LGS, NT, WAVE, K, K>;
  constexpr int lgGroups = LGS - K;
  constexpr int total = Map::total;
  constexpr int NI = Map::NI;
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int i = Map::item(tid, it);
    if ((total % NT) != 0 && i >= total) break;
    const int s = i >> lgGroups;
    const int g = i & ((1 << lgGroups) - 1);
    auto sd = W + (s << LGS);
    if (MODE == SIDES_DST || (MODE == SIDES_ALT && (s & 1)))
      tail_group<K, true>(sd, g, sec, SKIP0);
    else
      tail_group<K, false>(sd, g, sec, SKIP0);
  }
}

// Ends with the ordering before the next pass: the wave's own if NEXT_LOCAL
// and this pass stays in the wave's cells, else a workgroup barrier.
template <int K, int LO, int LGS, int NS, int NT, int WAVE, int MODE, bool SKIP0, bool NEXT_LOCAL,
          class Sync, class WSync, typename WP>
QFT_HD void bwd_chunk_s(WP W, int tid, Sync sync, WSync wsync) {
  using Map = PassMap<NS, LGS, NT, WAVE, K, LO + K - 1>;
  constexpr int R = 1 << K;
  constexpr int S = 1 << (LO + K - 1);
  constexpr int lgG = LO - 1;
  constexpr int G = 1 << lgG;
  constexpr int lgGroups = LGS - K;
  constexpr int total = Map::total;
  constexpr int NI = Map::NI;
  // the R <= 16 outputs of an item are a run inside one padding block (sides
  // start on a block boundary)
  static_assert(R <= kRowCells, "runs of at most one row unit");
  float2 y[NI][R];
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int i = Map::item(tid, it);
    if ((total % NT) != 0 && i >= total) break;
    const int s = i >> lgGroups;
    const int g = i & ((1 << lgGroups) - 1);
    const int j = g >> lgG, ii = g & (G - 1);
    auto sd = W + (s << LGS);
    const bool dst = MODE == SIDES_DST || (MODE == SIDES_ALT && (s & 1));
    if (SKIP0 && j == 0) {
      if (dst) bwd_head_load_s<K, true, 1, G>(sd, ii, y[it]);
      else bwd_head_load_s<K, false, 1, G>(sd, ii, y[it]);
    } else {
      if (dst) bwd_group_load_s<K, G, true>(sd, j * S, ii, y[it]);
      else bwd_group_load_s<K, G, false>(sd, j * S, ii, y[it]);
    }
  }
  pass_sync<Map::local>(sync, wsync);
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int i = Map::item(tid, it);
    if ((total % NT) != 0 && i >= total) break;
    const int s = i >> lgGroups;
    const int g = i & ((1 << lgGroups) - 1);
    const int j = g >> lgG, ii = g & (G - 1);
    auto sd = W + (s << LGS);
    if (SKIP0 && j == 0) {
      bwd_head_store_s<K, 1, G>(sd, ii, y[it]);
    } else {
      const auto r = pad_row(sd, j * S + ii * R);
#pragma unroll
      for (int e = 0; e < R; ++e) r.run(e) = y[it][e];
    }
  }
  pass_sync<Map::local && NEXT_LOCAL>(sync, wsync);
}

// Rounds per LDS pass (KC) of the forward and backward chunks, and fused
// innermost rounds (KT) of the tail.  A forward chunk of K rounds holds a
// closed group of 2^(K+1) cells in one thread, so KC = 3 with 16 cells per
// thread and KC = 4 with 32.  The tail takes KC + 1 rounds where that saves
// a pass (the rounds above it a multiple of KC), else KC.
template <int NS, int LGS, int NT>
QFT_HD constexpr int sweep_kc() {
  return ((NS << LGS) / NT) >= 32 ? 4 : 3;
}
QFT_HD constexpr int sweep_tail_rounds(int top, int kc) {
  return top <= kc ? top : ((top - kc - 1) % kc == 0 ? kc + 1 : kc);
}

// Whether the LDS pass that follows the forward chunk ending at round 2^HI
// (the next forward chunk, else the tail of KT rounds) stays in each wave's
// cells (PassMap).
template <int HI, int KT, int KC, int LGS, int NS, int NT, int WAVE>
QFT_HD constexpr bool fwd_next_local() {
  if constexpr (HI > KT) {
    constexpr int K = cmin<KC, HI - KT>::v;
    return PassMap<NS, LGS, NT, WAVE, K + 1, HI>::local;
  } else {
    return PassMap<NS, LGS, NT, WAVE, KT, KT>::local;
  }
}

// forward chunks for rounds (KT, HI], top down, each followed by the
// ordering the next pass needs
template <int HI, int KT, int KC, int LGS, int NS, int NT, int WAVE, int MODE, bool SKIP0,
          bool SF, class Sync, class WSync, typename WP>
QFT_HD void fwd_rounds_s(WP W, const float* sec, int tid, Sync sync, WSync wsync) {
  if constexpr (HI > KT) {
    constexpr int K = cmin<KC, HI - KT>::v;
    fwd_chunk_s<K, HI, LGS, NS, NT, WAVE, MODE, SKIP0, SF>(W, sec, tid);
    pass_sync<PassMap<NS, LGS, NT, WAVE, K + 1, HI>::local &&
              fwd_next_local<HI - K, KT, KC, LGS, NS, NT, WAVE>()>(sync, wsync);
    fwd_rounds_s<HI - K, KT, KC, LGS, NS, NT, WAVE, MODE, SKIP0, SF>(W, sec, tid, sync, wsync);
  }
}

// Whether the backward chunk starting at round 2^LO (if LO <= TOP) stays in
// each wave's cells; past the last chunk the caller's next stage does not.
template <int LO, int TOP, int KC, int LGS, int NS, int NT, int WAVE>
QFT_HD constexpr bool bwd_local() {
  if constexpr (LO <= TOP) {
    constexpr int K = cmin<KC, TOP - LO + 1>::v;
    return PassMap<NS, LGS, NT, WAVE, K, LO + K - 1>::local;
  } else {
    return false;
  }
}

// backward chunks for rounds [LO, TOP], bottom up; the last one ends with a
// workgroup barrier
template <int LO, int TOP, int KC, int LGS, int NS, int NT, int WAVE, int MODE, bool SKIP0,
          class Sync, class WSync, typename WP>
QFT_HD void bwd_rounds_s(WP W, int tid, Sync sync, WSync wsync) {
  if constexpr (LO <= TOP) {
    constexpr int K = cmin<KC, TOP - LO + 1>::v;
    bwd_chunk_s<K, LO, LGS, NS, NT, WAVE, MODE, SKIP0,
                bwd_local<LO + K, TOP, KC, LGS, NS, NT, WAVE>()>(W, tid, sync, wsync);
    bwd_rounds_s<LO + K, TOP, KC, LGS, NS, NT, WAVE, MODE, SKIP0>(W, tid, sync, wsync);
  }
}

// Forward rounds S = 2^TOP .. 2 and backward rounds back up (TOP >= 1).
// Expects a workgroup barrier before and ends with one; in between, passes
// whose segments fit one wave's cells are ordered by the wave alone.
template <int TOP, int LGS, int NS, int NT, int WAVE, int MODE, bool SKIP0, bool SF = false,
          class Sync, class WSync, typename WP>
QFT_HD void sweeps_s(WP W, const float* sec, int tid, Sync sync, WSync wsync) {
  if constexpr (TOP >= 1) {
    constexpr int KC = sweep_kc<NS, LGS, NT>();
    constexpr int KT = sweep_tail_rounds(TOP, KC);
    fwd_rounds_s<TOP, KT, KC, LGS, NS, NT, WAVE, MODE, SKIP0, SF>(W, sec, tid, sync, wsync);
    tail_chunk_s<KT, LGS, NS, NT, WAVE, MODE, SKIP0>(W, sec, tid);
    pass_sync<PassMap<NS, LGS, NT, WAVE, KT, KT>::local &&
              bwd_local<KT + 1, TOP, KC, LGS, NS, NT, WAVE>()>(sync, wsync);
    bwd_rounds_s<KT + 1, TOP, KC, LGS, NS, NT, WAVE, MODE, SKIP0>(W, tid, sync, wsync);
  }
}

// One chain level P = 2^p for T transforms of 2^LOGN cells (closed groups).
template <int p, int LOGN, int T, int NT, typename WP>
QFT_HD void chain_level_s(WP W, int tid) {
  constexpr int per_t = (p <= 2) ? 1 : 1 + 2 * (1 << (p - 3));
  constexpr int total = T * per_t;
  constexpr int NI = (total + NT - 1) / NT;
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int i = tid + it * NT;
    if ((total % NT) != 0 && i >= total) break;
    const int t = i / per_t;
    const int g = i - t * per_t;
    chain_item(W + (t << LOGN), LOGN, p, g);
  }
}

template <int p, int PHI, int LOGN, int T, int NT, class Sync, typename WP>
QFT_HD void chain_levels_s(WP W, int tid, Sync sync) {
  if constexpr (p <= PHI) {
    chain_level_s<p, LOGN, T, NT>(W, tid);
    sync();
    chain_levels_s<p + 1, PHI, LOGN, T, NT>(W, tid, sync);
  }
}

// Chain P = 2 .. 2^LOGN: small levels wave-synchronously (transform t on wave
// t % waves), the rest with workgroup barriers.
template <int LOGN, int T, int NT, int WAVE, class Sync, class WSync, typename WP>
QFT_HD void chain_s(WP W, int tid, Sync sync, WSync wsync) {
  constexpr int PW = cmin<9, LOGN>::v;
  constexpr int NW = (NT + WAVE - 1) / WAVE;
  constexpr int LANES = cmin<NT, WAVE>::v;
  constexpr int ROUNDS = (T + NW - 1) / NW;
  const int wave = tid / WAVE, lane = tid - wave * WAVE;
  for (int r = 0; r < ROUNDS; ++r) {
    const int t = wave + r * NW;
#pragma unroll
    for (int p = 1; p <= PW; ++p) {
      if (t < T) {
        const int per_t = chain_groups(p);
        for (int g = lane; g < per_t; g += LANES) chain_item(W + (t << LOGN), LOGN, p, g);
      }
      wsync();
    }
  }
  sync();
  chain_levels_s<PW + 1, LOGN, LOGN, T, NT>(W, tid, sync);
}

// ===========================================================================
// Fused DCT-0 / DST-0 chain (the backward half of ``dct``/``dst``, eqs.
// qft_5C, qft_5D, qft_6), several levels per LDS round trip.
//
// Level Q = 2^q of the DCT chain takes E(i) = D_{Q/2}(i), i in [0, Q/4]
// (cell i; E(Q/4) in the top cell) and the DCT-II block O(i), i < Q/4 (cell
// Q/4 + i) to D_Q(i) = E(i) + O(i), D_Q(Q/2 - i) = E(i) - O(i) (i < Q/4) and
// D_Q(Q/4) = E(Q/4); D_Q(i) goes to cell i, D_Q(Q/2) to the top cell.  Level
// Q of the DST chain takes E(i) = S_{Q/2}(i), i in [1, Q/4) (cell i) and the
// DST-II block O(i), i in [1, Q/4] (cell Q/4 + i - 1) to S_Q(i) = E(i) + O(i),
// S_Q(Q/2 - i) = O(i) - E(i) and S_Q(Q/4) = O(Q/4), S_Q(i) to cell i.
//
// An index i of level Q feeds the outputs i and Q/2 - i.  Followed from one
// input index k through K levels P, 2P, .., 2^(K-1) P, it gives 2^K outputs.
// For 1 <= k < P/4 the index stays below Q/4 at every level Q, and output m
// has index c_m + s_m k with compile-time c_m and s_m = +-1, the same on the
// DCT and the DST side ("generic group" k).  Group 0 takes what is left: on
// the DCT side index 0 together with the top cell (an index equal to Q/4
// passes level Q unchanged, index 0 produces the next top Q/2), 2^K + 1
// outputs; on the DST side the indices Q/4 that each level adds from O(Q/4),
// 2^K - 1 outputs.  A pass over K levels is therefore P/4 independent groups
// per side, each loading and storing its cells once.
// ===========================================================================

// Index constant and sign of output m of a generic group after a levels
// (bit a-1-l of m selects the second output Q/2 - i of level l).
QFT_HD constexpr int chain_c(int P, int a, int m) {
  int c = 0;
  for (int l = 0; l < a; ++l)
    if ((m >> (a - 1 - l)) & 1) c = ((P << l) >> 1) - c;
  return c;
}
QFT_HD constexpr int chain_sgn(int a, int m) {
  int s = 1;
  for (int l = 0; l < a; ++l)
    if ((m >> (a - 1 - l)) & 1) s = -s;
  return s;
}

// Index list of group 0 after a levels starting at P (DCT: index 0 and the
// top index P/4 to begin with; DST: empty, one index added per level).
struct ChainList {
  int n;
  int idx[40];
};

QFT_HD constexpr ChainList chain_special(int P, int a, bool dst) {
  ChainList L{};
  if (!dst) {
    L.n = 2;
    L.idx[0] = 0;
    L.idx[1] = P / 4;
  }
  for (int l = 0; l < a; ++l) {
    const int Q = P << l;
    ChainList N{};
    for (int m = 0; m < L.n; ++m) {
      const int i = L.idx[m];
      if (dst || i < Q / 4) {
        N.idx[N.n++] = i;
        N.idx[N.n++] = Q / 2 - i;
      } else {
        N.idx[N.n++] = i;
      }
    }
    if (dst) N.idx[N.n++] = Q / 4;
    L = N;
  }
  return L;
}

// For output m of the DCT group 0 after K levels: the DST group-0 output with
// the same index, or -1 (indices 0 and Q/2, which have no DST partner).
struct ChainPairing {
  int ms[40];
};

QFT_HD constexpr ChainPairing chain_pairing(int P, int K) {
  ChainPairing r{};
  const ChainList d = chain_special(P, K, false);
  const ChainList s = chain_special(P, K, true);
  for (int m = 0; m < d.n; ++m) {
    r.ms[m] = -1;
    for (int q = 0; q < s.n; ++q)
      if (s.idx[q] == d.idx[m]) r.ms[m] = q;
  }
  return r;
}

// Generic group k (1 <= k < P/4): loads E(k) and the 2^K - 1 block values it
// meets, returns the 2^K outputs in v (output m has index c_m + s_m k).
template <int P, int K, bool DST, typename SP>
QFT_HD void chain_generic(SP sd, int k, float2* v) {
  float2 o[1 << K];
  if constexpr ((P / 4) % kRowCells == 0) {
    // every index is a multiple C >= P/4 of P/4 plus k or -k: rows at k and
    // P/4 - k (both >= 0)
    constexpr int A = P / 4;
    const auto rp = pad_row(sd, k - (DST ? 1 : 0));
    const auto rm = pad_row(sd, A - k - (DST ? 1 : 0));
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int Q4 = (P << l) >> 2;
#pragma unroll
      for (int m = 0; m < (1 << l); ++m) {
        const int C = Q4 + chain_c(P, l, m);
        o[(1 << l) - 1 + m] = chain_sgn(l, m) > 0 ? (float2)rp[C] : (float2)rm[C - A];
      }
    }
  } else {
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int Q4 = (P << l) >> 2;
#pragma unroll
      for (int m = 0; m < (1 << l); ++m)
        o[(1 << l) - 1 + m] = sd[Q4 + chain_c(P, l, m) + chain_sgn(l, m) * k - (DST ? 1 : 0)];
    }
  }
  v[0] = sd[k];
#pragma unroll
  for (int l = 0; l < K; ++l) {
#pragma unroll
    for (int m = (1 << l) - 1; m >= 0; --m) {
      const float2 E = v[m], O = o[(1 << l) - 1 + m];
      v[2 * m] = cadd(E, O);
      v[2 * m + 1] = DST ? csub(O, E) : csub(E, O);
    }
  }
}

template <int P, int K, typename SP>
QFT_HD void chain_generic_store(SP sd, int k, const float2* v) {
  if constexpr ((P / 2) % kRowCells == 0) {
    // output indices: multiples of P/2 plus k, or multiples C >= P/2 minus k:
    // rows at k and P/2 - k (both >= 0)
    constexpr int A = P / 2;
    const auto rp = pad_row(sd, k);
    const auto rm = pad_row(sd, A - k);
#pragma unroll
    for (int m = 0; m < (1 << K); ++m) {
      if (chain_sgn(K, m) > 0) rp[chain_c(P, K, m)] = v[m];
      else rm[chain_c(P, K, m) - A] = v[m];
    }
  } else {
#pragma unroll
    for (int m = 0; m < (1 << K); ++m) sd[chain_c(P, K, m) + chain_sgn(K, m) * k] = v[m];
  }
}

// Group 0 of one side, levels L .. K-1 of the pass (v holds the list of
// level L in the order of chain_special).
template <int P, int K, int L, bool DST, typename SP>
QFT_HD void chain_special_levels(SP sd, float2* v) {
  if constexpr (L < K) {
    constexpr ChainList cur = chain_special(P, L, DST);
    constexpr ChainList nxt = chain_special(P, L + 1, DST);
    constexpr int Q = P << L;
    float2 nv[(1 << K) + 1];
    int pos = 0;
#pragma unroll
    for (int m = 0; m < cur.n; ++m) {
      const int i = cur.idx[m];
      if (DST || i < Q / 4) {
        const float2 E = v[m], O = sd[Q / 4 + i - (DST ? 1 : 0)];
        nv[pos] = cadd(E, O);
        nv[pos + 1] = DST ? csub(O, E) : csub(E, O);
        pos += 2;
      } else {
        nv[pos] = v[m];
        pos += 1;
      }
    }
    if constexpr (DST) nv[nxt.n - 1] = sd[Q / 2 - 1];  // S_Q(Q/4) = O(Q/4)
#pragma unroll
    for (int m = 0; m < nxt.n; ++m) v[m] = nv[m];
    chain_special_levels<P, K, L + 1, DST>(sd, v);
  }
}

template <int P, int K, bool DST, typename SP>
QFT_HD void chain_special_load(SP sd, SP top, float2* v) {
  if constexpr (!DST) {
    v[0] = sd[0];
    v[1] = *top;
  }
  chain_special_levels<P, K, 0, DST>(sd, v);
}

template <int P, int K, bool DST, typename SP>
QFT_HD void chain_special_store(SP sd, SP top, const float2* v) {
  constexpr ChainList fin = chain_special(P, K, DST);
  constexpr int half = (P << (K - 1)) >> 1;  // Q/2 of the last level
#pragma unroll
  for (int m = 0; m < fin.n; ++m) {
    const int i = fin.idx[m];
    if (!DST && i == half) *top = v[m];
    else sd[i] = v[m];
  }
}

// Side pointers of transform t: DCT side, DST side, top cell.
template <typename WP>
struct TileSides {
  WP W;
  int logn;
  QFT_HD WP dc(int t) const { return W + (t << logn); }
  QFT_HD WP ds(int t) const { return W + (t << logn) + (1 << (logn - 1)); }
  QFT_HD WP top(int t) const { return ds(t); }
};

// One pass: levels P .. 2^(K-1) P of both sides of transforms [0, T); item =
// (transform, group) with the DCT and the DST group of the same index, over
// NT threads.  All loads, then `sync`, then all stores, then `sync`.
template <int P, int K, int T, int NT, class Sync, class Acc>
QFT_HD void chain_pass(const Acc& acc, int tid, bool active, Sync sync) {
  constexpr int G = P / 4;
  constexpr int total = T * G;
  constexpr int NI = (total + NT - 1) / NT;
  constexpr int S = (1 << K) + 1;
  float2 vc[NI][S], vs[NI][S];
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int i = tid + it * NT;
    if (active && i < total) {
      const int t = i / G, g = i - t * G;
      if (g == 0) {
        chain_special_load<P, K, false>(acc.dc(t), acc.top(t), vc[it]);
        chain_special_load<P, K, true>(acc.ds(t), acc.top(t), vs[it]);
      } else {
        chain_generic<P, K, false>(acc.dc(t), g, vc[it]);
        chain_generic<P, K, true>(acc.ds(t), g, vs[it]);
      }
    }
  }
  sync();
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int i = tid + it * NT;
    if (active && i < total) {
      const int t = i / G, g = i - t * G;
      if (g == 0) {
        chain_special_store<P, K, false>(acc.dc(t), acc.top(t), vc[it]);
        chain_special_store<P, K, true>(acc.ds(t), acc.top(t), vs[it]);
      } else {
        chain_generic_store<P, K>(acc.dc(t), g, vc[it]);
        chain_generic_store<P, K>(acc.ds(t), g, vs[it]);
      }
    }
  }
  sync();
}

// Levels 1 .. B of one side in one thread (B >= 1; DCT base P = 2 is
// (c(0) + c(N/2), c(0) - c(N/2)), DST base P = 4 is the identity).
template <int B, typename SP>
QFT_HD void chain_base_dct(SP sd, SP top) {
  constexpr int NV = (1 << (B - 1)) + 1;
  float2 D[NV], in[NV];
#pragma unroll
  for (int c = 0; c < NV - 1; ++c) in[c] = sd[c];
  const float2 ct = *top;
  D[0] = cadd(in[0], ct);
  D[1] = csub(in[0], ct);
#pragma unroll
  for (int q = 2; q <= B; ++q) {
    const int Q = 1 << q;
    float2 nd[NV];
#pragma unroll
    for (int i = 0; i < Q / 4; ++i) {
      const float2 O = in[Q / 4 + i];
      nd[i] = cadd(D[i], O);
      nd[Q / 2 - i] = csub(D[i], O);
    }
    nd[Q / 4] = D[Q / 4];
#pragma unroll
    for (int i = 0; i <= Q / 2; ++i) D[i] = nd[i];
  }
#pragma unroll
  for (int c = 0; c < NV - 1; ++c) sd[c] = D[c];
  *top = D[NV - 1];
}

template <int B, typename SP>
QFT_HD void chain_base_dst(SP sd) {
  if constexpr (B >= 3) {
    constexpr int NV = 1 << (B - 1);
    float2 Sv[NV], in[NV];
#pragma unroll
    for (int c = 1; c < NV; ++c) in[c] = sd[c];
    Sv[1] = in[1];
#pragma unroll
    for (int q = 3; q <= B; ++q) {
      const int Q = 1 << q;
      float2 ns[NV];
#pragma unroll
      for (int i = 1; i < Q / 4; ++i) {
        const float2 O = in[Q / 4 + i - 1];
        ns[i] = cadd(Sv[i], O);
        ns[Q / 2 - i] = csub(O, Sv[i]);
      }
      ns[Q / 4] = in[Q / 2 - 1];
#pragma unroll
      for (int i = 1; i < Q / 2; ++i) Sv[i] = ns[i];
    }
#pragma unroll
    for (int c = 1; c < NV; ++c) sd[c] = Sv[c];
  }
}

// Global input and output of the transforms of a tile.  A tile body asks its
// IO for two things:
//  * fetch(t, m, r) / fold(r, m, lo, hi): the samples of position m of
//    transform t (0 <= m < N/2) and the two heap values they give: for
//    m >= 1 the DCT-side cell c(m) and the DST-side cell d(m) of the real fold
//    (Sec. 4.2), for m = 0 the cells c(0) and c(N/2);
//  * put(o, n, k, C, S) for 0 < k < N/2 and put_edge(o, k, C) for k = 0, N/2:
//    the outputs from the DCT-0 result C(k) and the DST-0 result S(k).
// Every cell carries two real signals (the float2 lanes).
//
// ContigIO / GatherIO: complex transforms, lane x = Re, lane y = Im (cdft,
// Sec. 4.1): X(k) = C(k) - i S(k) per real signal, combined into
// X(k), X(N-k).  SWAP exchanges real and imaginary parts on every load and
// store, which turns the forward transform into the adjoint:
// F^H g = swap(F swap(g)).  Transform t starts at x + t 2^LOGN (contiguous
// batch) or at x + offs[t] (an uneven batch's offset list).
template <int DT, bool SWAP>
struct ComplexIO {
  using E = typename Store<DT>::T;
  struct Raw {
    float2 a, b;
  };
  QFT_HD static float2 load(const E* p, int i) { return sw<SWAP>(Store<DT>::ld(p, i)); }
  QFT_HD static void store(E* p, int i, float2 v) { Store<DT>::st(p, i, sw<SWAP>(v)); }
  QFT_HD static void fold(const Raw& r, int m, float2& lo, float2& hi) {
    if (m == 0) {
      lo = r.a;
      hi = r.b;
    } else {
      lo = cadd(r.a, r.b);
      hi = csub(r.a, r.b);
    }
  }
  QFT_HD static void put(E* Xt, int n, int k, float2 C, float2 S) {
    store(Xt, k, make_float2(C.x + S.y, C.y - S.x));
    store(Xt, n - k, make_float2(C.x - S.y, C.y + S.x));
  }
  QFT_HD static void put_edge(E* Xt, int k, float2 C) { store(Xt, k, C); }
};

template <int DT, bool SWAP, int LOGN>
struct ContigIO : ComplexIO<DT, SWAP> {
  using E = typename Store<DT>::T;
  using typename ComplexIO<DT, SWAP>::Raw;
  const E* x;
  E* X;
  QFT_HD ContigIO(const E* x_, E* X_) : x(x_), X(X_) {}
  QFT_HD E* out(int t) const { return X + ((int64_t)t << LOGN); }
  QFT_HD void fetch(int t, int m, Raw& r) const {
    constexpr int n = 1 << LOGN, h = n >> 1;
    const E* xt = x + ((int64_t)t << LOGN);
    r.a = this->load(xt, m);
    r.b = this->load(xt, m == 0 ? h : n - m);
  }
};

template <int DT, bool SWAP>
struct GatherIO : ComplexIO<DT, SWAP> {
  using E = typename Store<DT>::T;
  using typename ComplexIO<DT, SWAP>::Raw;
  const E* x;
  E* X;
  const int64_t* offs;
  int logn;
  QFT_HD GatherIO(const E* x_, E* X_, const int64_t* o, int lg)
      : x(x_), X(X_), offs(o), logn(lg) {}
  QFT_HD E* out(int t) const { return X + offs[t]; }
  QFT_HD void fetch(int t, int m, Raw& r) const {
    const int n = 1 << logn, h = n >> 1;
    const E* xt = x + offs[t];
    r.a = this->load(xt, m);
    r.b = this->load(xt, m == 0 ? h : n - m);
  }
};

// Contiguous batch of transforms of a run-time length 2^logn (multi-pass).
template <int DT, bool SWAP>
struct ContigRtIO : ComplexIO<DT, SWAP> {
  using E = typename Store<DT>::T;
  using typename ComplexIO<DT, SWAP>::Raw;
  const E* x;
  E* X;
  int logn;
  QFT_HD ContigRtIO(const E* x_, E* X_, int lg) : x(x_), X(X_), logn(lg) {}
  QFT_HD E* out(int t) const { return X + ((int64_t)t << logn); }
  QFT_HD void fetch(int t, int m, Raw& r) const {
    const int n = 1 << logn, h = n >> 1;
    const E* xt = x + ((int64_t)t << logn);
    r.a = this->load(xt, m);
    r.b = this->load(xt, m == 0 ? h : n - m);
  }
};

// Real-input transform (rdft, Sec. 4.2) of real signals 2t and 2t+1 of a
// batch of `rows` signals of N = 2^LOGN points (row r at x + r N), as the
// two lanes of transform t.  Output: the half spectrum X(k) = C(k) - i S(k),
// k = 0..N/2, of each signal (row r at X + r (N/2 + 1)).  Signal 2t+1 past
// the batch reads as zero and is not written.
template <int DT, int LOGN>
struct RealPairIO {
  using R = typename RStore<DT>::T;
  using E = typename Store<DT>::T;
  struct Raw {
    float2 a, b;
  };
  struct Out {
    E* A;
    E* B;
  };
  const R* x;
  E* X;
  int64_t rows;
  int lg = LOGN;  // log2 N: the template's, or given at run time when LOGN = 0
  QFT_HD int nn() const { return LOGN ? (1 << LOGN) : (1 << lg); }
  QFT_HD bool has_b(int t) const { return 2 * (int64_t)t + 1 < rows; }
  QFT_HD float2 pair(int t, int i) const {
    const int64_t r0 = 2 * (int64_t)t;
    const float va = RStore<DT>::ld(x, r0 * nn() + i);
    const float vb = has_b(t) ? RStore<DT>::ld(x, (r0 + 1) * nn() + i) : 0.f;
    return make_float2(va, vb);
  }
  QFT_HD void fetch(int t, int m, Raw& r) const {
    const int n = nn(), h = n >> 1;
    r.a = pair(t, m);
    r.b = pair(t, m == 0 ? h : n - m);
  }
  QFT_HD static void fold(const Raw& r, int m, float2& lo, float2& hi) {
    ComplexIO<DT, false>::fold(typename ComplexIO<DT, false>::Raw{r.a, r.b}, m, lo, hi);
  }
  QFT_HD Out out(int t) const {
    const int64_t r0 = 2 * (int64_t)t, h = nn() >> 1;
    return Out{X + r0 * (h + 1), has_b(t) ? X + (r0 + 1) * (h + 1) : nullptr};
  }
  QFT_HD static void put(const Out& o, int, int k, float2 C, float2 S) {
    Store<DT>::st(o.A, k, make_float2(C.x, -S.x));
    if (o.B) Store<DT>::st(o.B, k, make_float2(C.y, -S.y));
  }
  QFT_HD static void put_edge(const Out& o, int k, float2 C) {
    Store<DT>::st(o.A, k, make_float2(C.x, 0.f));
    if (o.B) Store<DT>::st(o.B, k, make_float2(C.y, 0.f));
  }
};

// Standalone DCT-0 and DST-0 of periodization N = 2^LOGN (``dct`` on
// s_dc_tt, eq. qft_0B; ``dst`` on s_ds_tt, eq. qft_0C): inputs c(n),
// n = 0..N/2 (row r at c + r (N/2+1)) and d(n), n = 1..N/2-1 (row r at
// d + r (N/2-1), d(n) at index n-1); outputs C(k), k = 0..N/2 and S(k),
// k = 1..N/2-1 in the same layouts.  Signals 2t and 2t+1 are the lanes of
// transform t.  A null input pair (c and C, or d and S) reads as zero and is
// not written.
template <int DT, int LOGN>
struct DctDstIO {
  using R = typename RStore<DT>::T;
  struct Raw {
    float2 a, b;
  };
  struct Out {
    R* CA;
    R* CB;
    R* SA;
    R* SB;
  };
  const R* c;
  const R* d;
  R* C;
  R* S;
  int64_t rows;
  int lg = LOGN;  // log2 N: the template's, or given at run time when LOGN = 0
  QFT_HD int nn() const { return LOGN ? (1 << LOGN) : (1 << lg); }
  QFT_HD bool has_b(int t) const { return 2 * (int64_t)t + 1 < rows; }
  QFT_HD float2 pair(const R* p, int len, int t, int i) const {
    if (!p) return make_float2(0.f, 0.f);
    const int64_t r0 = 2 * (int64_t)t;
    const float va = RStore<DT>::ld(p, r0 * len + i);
    const float vb = has_b(t) ? RStore<DT>::ld(p, (r0 + 1) * len + i) : 0.f;
    return make_float2(va, vb);
  }
  QFT_HD void fetch(int t, int m, Raw& r) const {
    const int h = nn() >> 1;
    if (m == 0) {
      r.a = pair(c, h + 1, t, 0);
      r.b = pair(c, h + 1, t, h);
    } else {
      r.a = pair(c, h + 1, t, m);
      r.b = pair(d, h - 1, t, m - 1);
    }
  }
  QFT_HD static void fold(const Raw& r, int, float2& lo, float2& hi) {
    lo = r.a;
    hi = r.b;
  }
  QFT_HD Out out(int t) const {
    const int64_t r0 = 2 * (int64_t)t, h = nn() >> 1;
    const bool b = has_b(t);
    return Out{C ? C + r0 * (h + 1) : nullptr, (C && b) ? C + (r0 + 1) * (h + 1) : nullptr,
               S ? S + r0 * (h - 1) : nullptr, (S && b) ? S + (r0 + 1) * (h - 1) : nullptr};
  }
  QFT_HD static void put(const Out& o, int, int k, float2 Cv, float2 Sv) {
    if (o.CA) RStore<DT>::st(o.CA, k, Cv.x);
    if (o.CB) RStore<DT>::st(o.CB, k, Cv.y);
    if (o.SA) RStore<DT>::st(o.SA, k - 1, Sv.x);
    if (o.SB) RStore<DT>::st(o.SB, k - 1, Sv.y);
  }
  QFT_HD static void put_edge(const Out& o, int k, float2 Cv) {
    if (o.CA) RStore<DT>::st(o.CA, k, Cv.x);
    if (o.CB) RStore<DT>::st(o.CB, k, Cv.y);
  }
};

struct NoIO {};

// Transforms [t0, t0 + T') of an accessor, as an accessor of their own.
template <class Acc>
struct ChainSub {
  Acc a;
  int t0;
  QFT_HD auto dc(int t) const { return a.dc(t0 + t); }
  QFT_HD auto ds(int t) const { return a.ds(t0 + t); }
  QFT_HD auto top(int t) const { return a.top(t0 + t); }
};

// Levels 1 .. B of the base: one thread per (transform, side).
template <int B, int T, int NT, class Acc>
QFT_HD void chain_base(const Acc& acc, int tid, bool active) {
  constexpr int total = 2 * T;
#pragma unroll
  for (int it = 0; it < (total + NT - 1) / NT; ++it) {
    const int i = tid + it * NT;
    if (active && i < total) {
      const int t = i >> 1;
      if (i & 1) chain_base_dst<B>(acc.ds(t));
      else chain_base_dct<B>(acc.dc(t), acc.top(t));
    }
  }
}

// Passes of three levels starting at level PL while PL < PEND, over T
// transforms and NT threads ordered by `sync`.
template <int PL, int PEND, int T, int NT, class Sync, class Acc>
QFT_HD void chain_passes(const Acc& acc, int tid, bool active, Sync sync) {
  if constexpr (PL < PEND) {
    chain_pass<(1 << PL), 3, T, NT>(acc, tid, active, sync);
    chain_passes<PL + 3, PEND, T, NT>(acc, tid, active, sync);
  }
}

// First pass level (>= PL, in steps of 3, below PEND) whose items per wave
// exceed the wave's lanes.
QFT_HD constexpr int chain_first_block_pass(int pl, int pend, int tpw, int lanes) {
  return (pl >= pend || tpw * ((1 << pl) / 4) > lanes)
             ? pl
             : chain_first_block_pass(pl + 3, pend, tpw, lanes);
}

// Last pass (levels PLOG-2 .. PLOG) fused with the cdft combine of Sec. 4.1:
// the DCT and the DST group of one index hold C and S at the same indices.
template <int PLOG, int T, int NT, class Acc, class IO>
QFT_HD void chain_top_combine(const Acc& acc, const IO& io, int Tact, int tid) {
  constexpr int N = 1 << PLOG, P = N / 4, G = P / 4, K = 3;
  constexpr int total = T * G;
  constexpr int S = (1 << K) + 1;
#pragma unroll
  for (int it = 0; it < (total + NT - 1) / NT; ++it) {
    const int i = tid + it * NT;
    if (i < total) {
      const int t = i / G, g = i - t * G;
      if (t < Tact) {
        const auto Xt = io.out(t);
        float2 vc[S], vs[S];
        if (g == 0) {
          chain_special_load<P, K, false>(acc.dc(t), acc.top(t), vc);
          chain_special_load<P, K, true>(acc.ds(t), acc.top(t), vs);
          constexpr ChainList fin = chain_special(P, K, false);
          constexpr ChainPairing pr = chain_pairing(P, K);
#pragma unroll
          for (int m = 0; m < fin.n; ++m) {
            if (pr.ms[m] < 0) io.put_edge(Xt, fin.idx[m], vc[m]);  // k = 0, N/2
            else io.put(Xt, N, fin.idx[m], vc[m], vs[pr.ms[m]]);
          }
        } else {
          chain_generic<P, K, false>(acc.dc(t), g, vc);
          chain_generic<P, K, true>(acc.ds(t), g, vs);
#pragma unroll
          for (int m = 0; m < (1 << K); ++m)
            io.put(Xt, N, chain_c(P, K, m) + chain_sgn(K, m) * g, vc[m], vs[m]);
        }
      }
    }
  }
}

// Base levels of a chain of PLOG levels: the rest is a whole number of
// three-level passes, the last one starting at PLOG - 2.
QFT_HD constexpr int chain_base_levels(int plog) {
  return plog <= 4 ? plog : ((plog - 3) % 3 == 0 ? 3 : ((plog - 3) % 3 == 1 ? 4 : 2));
}

// Levels 1 .. PLOG of T transforms (PLOG >= 5): levels 1..B, then passes of
// three levels.  The base and the passes with at most one item per lane run
// per wavefront (wave w owns transforms [w TPW, (w+1) TPW), ordered by
// `wsync`); the others use the whole workgroup.  COMBINE: the last pass
// writes X(k), X(N-k) for t < Tact to X instead of the side cells and ends
// without a barrier (the caller synchronises before it reuses the LDS).
template <int PLOG, int T, int NT, int WAVE, bool COMBINE, class Sync, class WSync, class Acc,
          class IO>
QFT_HD void chain_fused(const Acc& acc, const IO& io, int Tact, int tid, Sync sync, WSync wsync) {
  static_assert(PLOG >= 5, "the fused chain starts at N = 32");
  constexpr int B = chain_base_levels(PLOG);
  constexpr int LANES = NT < WAVE ? NT : WAVE;
  constexpr int NW = NT / LANES;
  constexpr int TPW = (T + NW - 1) / NW;
  constexpr int PTOP = PLOG - 2;
  constexpr int PBLK = chain_first_block_pass(B + 1, PTOP, TPW, LANES);
  static_assert(2 * TPW <= LANES, "base items exceed one wavefront");
  const int w = tid / LANES, lane = tid - w * LANES;
  const bool wact = w * TPW < T;
  const ChainSub<Acc> sub{acc, w * TPW};
  chain_base<B, TPW, LANES>(sub, lane, wact);
  wsync();
  chain_passes<B + 1, PBLK, TPW, LANES>(sub, lane, wact, wsync);
  sync();
  chain_passes<PBLK, PTOP, T, NT>(acc, tid, true, sync);
  if constexpr (COMBINE) chain_top_combine<PLOG, T, NT>(acc, io, Tact, tid);
  else chain_pass<(1 << PTOP), 3, T, NT>(acc, tid, true, sync);
}

// ---------------------------------------------------------------------------
// Chain passes of the multi-pass path: levels P = 2^p .. 2^(p+K-1) (P >= 8)
// with p known at run time.  Every index of a K-level group is a multiple of
// P/4 plus 0 or +-k, so the groups of chain_generic / chain_special_load are
// evaluated on the index sets of P = 4 scaled by u = P/4.  E values (cells
// [0, P/4) of each side, E(P/4) in the top cell) come from one buffer, the
// DCT-II / DST-II blocks from another.
// ---------------------------------------------------------------------------
template <int K, bool DST, typename EP, typename OP>
QFT_HD void chain_generic_rt(EP se, OP so, int u, int k, float2* v) {
  float2 o[1 << K];
#pragma unroll
  for (int l = 0; l < K; ++l) {
#pragma unroll
    for (int m = 0; m < (1 << l); ++m)
      o[(1 << l) - 1 + m] =
          so[((1 << l) + chain_c(4, l, m)) * u + chain_sgn(l, m) * k - (DST ? 1 : 0)];
  }
  v[0] = se[k];
#pragma unroll
  for (int l = 0; l < K; ++l) {
#pragma unroll
    for (int m = (1 << l) - 1; m >= 0; --m) {
      const float2 E = v[m], O = o[(1 << l) - 1 + m];
      v[2 * m] = cadd(E, O);
      v[2 * m + 1] = DST ? csub(O, E) : csub(E, O);
    }
  }
}

template <int K, int L, bool DST, typename OP>
QFT_HD void chain_special_levels_rt(OP so, int u, float2* v) {
  if constexpr (L < K) {
    constexpr ChainList cur = chain_special(4, L, DST);
    constexpr ChainList nxt = chain_special(4, L + 1, DST);
    constexpr int Qn = 4 << L;
    float2 nv[(1 << K) + 1];
    int pos = 0;
#pragma unroll
    for (int m = 0; m < cur.n; ++m) {
      const int i = cur.idx[m];
      if (DST || i < Qn / 4) {
        const float2 E = v[m], O = so[(Qn / 4 + i) * u - (DST ? 1 : 0)];
        nv[pos] = cadd(E, O);
        nv[pos + 1] = DST ? csub(O, E) : csub(E, O);
        pos += 2;
      } else {
        nv[pos] = v[m];
        pos += 1;
      }
    }
    if constexpr (DST) nv[nxt.n - 1] = so[(Qn / 2) * u - 1];  // S_Q(Q/4) = O(Q/4)
#pragma unroll
    for (int m = 0; m < nxt.n; ++m) v[m] = nv[m];
    chain_special_levels_rt<K, L + 1, DST>(so, u, v);
  }
}

// Loads and runs the K levels of group k of transform heap t: vc / vs get
// the DCT and DST outputs (generic: 2^K each; k = 0: the lists of
// chain_special(4, K, .), indices scaled by u).
template <int K, typename EP, typename OP>
QFT_HD void mp_chain_group(EP Et, OP Ot, int h, int u, int k, float2* vc, float2* vs) {
  if (k == 0) {
    vc[0] = Et[0];
    vc[1] = Et[h];  // top cell
    chain_special_levels_rt<K, 0, false>(Ot, u, vc);
    chain_special_levels_rt<K, 0, true>(Ot + h, u, vs);
  } else {
    chain_generic_rt<K, false>(Et, Ot, u, k, vc);
    chain_generic_rt<K, true>(Et + h, Ot + h, u, k, vs);
  }
}

// Chain pass, item i < batch * P/4 = (transform t, group k): E from Ein,
// blocks from Wo, outputs to Wout.  Ein == Wout is race free: group k reads
// the E cells k (k = 0: cell 0 and the top cell) and writes cell k, the top
// cell (k = 0) and cells >= P/4, which no other group reads.
template <int K, typename EP, typename OP, typename WP>
QFT_HD void mp_chain_item(EP Ein, OP Wo, WP Wout, int logn, int p, int64_t i) {
  const int h = 1 << (logn - 1), u = 1 << (p - 2);
  const int64_t b = (i >> (p - 2)) << logn;
  const int k = (int)(i & (u - 1));
  float2 vc[(1 << K) + 1], vs[(1 << K) + 1];
  mp_chain_group<K>(Ein + b, Wo + b, h, u, k, vc, vs);
  auto dc = Wout + b;
  auto ds = Wout + b + h;
  if (k == 0) {
    constexpr ChainList fc = chain_special(4, K, false);
    constexpr ChainList fs = chain_special(4, K, true);
    constexpr int half = 1 << K;  // Q/2 of the last level, scaled
#pragma unroll
    for (int m = 0; m < fc.n; ++m) dc[fc.idx[m] == half ? h : fc.idx[m] * u] = vc[m];
#pragma unroll
    for (int m = 0; m < fs.n; ++m) ds[fs.idx[m] * u] = vs[m];
  } else {
#pragma unroll
    for (int m = 0; m < (1 << K); ++m) {
      const int c = chain_c(4, K, m) * u + chain_sgn(K, m) * k;
      dc[c] = vc[m];
      ds[c] = vs[m];
    }
  }
}

// Last chain pass (its top level is N) fused with the combine of Sec. 4.1:
// C(k) and S(k) of one index meet in the DCT and the DST group of one item.
template <int K, class IO, typename EP, typename OP>
QFT_HD void mp_chain_combine_item(const IO& io, EP Ein, OP Wo, int logn, int p, int64_t i) {
  const int n = 1 << logn, h = n >> 1, u = 1 << (p - 2);
  const int64_t t = i >> (p - 2);
  const int64_t b = t << logn;
  const int k = (int)(i & (u - 1));
  float2 vc[(1 << K) + 1], vs[(1 << K) + 1];
  mp_chain_group<K>(Ein + b, Wo + b, h, u, k, vc, vs);
  const auto o = io.out((int)t);
  if (k == 0) {
    constexpr ChainList fc = chain_special(4, K, false);
    constexpr ChainPairing pr = chain_pairing(4, K);
#pragma unroll
    for (int m = 0; m < fc.n; ++m) {
      if (pr.ms[m] < 0) io.put_edge(o, fc.idx[m] * u, vc[m]);  // k = 0, N/2
      else io.put(o, n, fc.idx[m] * u, vc[m], vs[pr.ms[m]]);
    }
  } else {
#pragma unroll
    for (int m = 0; m < (1 << K); ++m)
      io.put(o, n, chain_c(4, K, m) * u + chain_sgn(K, m) * k, vc[m], vs[m]);
  }
}

// An opaque copy: the compiler must treat v as changed here (no instruction
// is emitted on the GPU).
QFT_HD void launder(int& v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(v));
#else
  (void)v;
#endif
}

// Whole tile: T transforms of 2^LOGN points, NT threads (LOGN >= 1), in
// three steps: tile_fetch_s loads a thread's fold items from x into
// registers, tile_fold_s folds them into LDS, tile_rest_s runs the rounds,
// the chain and the combine and writes X.  Fold item it of a thread is the
// pair (m, N - m) of transform t; the pair goes to heap cell
// (N >> (l + 2)) + (m >> (l + 1)), l = ctz(m), of both sides (m = 0: cells
// 0 and N/2).  With h = N/2 >= NT, t = it NT / h and m = tid + (it NT mod h);
// else every item of a thread has m = tid mod h and t steps by NT / h.
template <int LOGN, int T, int NT>
QFT_HD constexpr int tile_items() {
  static_assert(((T << (LOGN - 1)) % NT) == 0, "fold items per thread");
  return (T << (LOGN - 1)) / NT;
}

template <int LOGN, int T, int NT, class IO>
QFT_HD void tile_fetch_s(const IO& io, int Tact, int tid,
                         typename IO::Raw (&raw)[tile_items<LOGN, T, NT>()]) {
  constexpr int h = (1 << LOGN) >> 1;
  constexpr int FI = tile_items<LOGN, T, NT>();
  if constexpr (h >= NT) {
#pragma unroll
    for (int it = 0; it < FI; ++it) {
      const int t = (it * NT) / h;
      if (t < Tact) io.fetch(t, tid + (it * NT) % h, raw[it]);
    }
  } else {
    constexpr int TS = NT / h;
    const int m = tid & (h - 1);
    const int t0 = tid >> (LOGN - 1);
#pragma unroll
    for (int it = 0; it < FI; ++it)
      if (t0 + it * TS < Tact) io.fetch(t0 + it * TS, m, raw[it]);
  }
}

template <int LOGN, int T, int NT, typename WP, class IO>
QFT_HD void tile_fold_s(const IO& io, WP W, int Tact, int tid,
                        const typename IO::Raw (&raw)[tile_items<LOGN, T, NT>()]) {
  constexpr int n = 1 << LOGN, h = n >> 1;
  constexpr int FI = tile_items<LOGN, T, NT>();
  if constexpr (h >= NT) {
    // for tid != 0 the low bits of m, hence l, are tid's, and the cell is a
    // per-thread base plus a constant shifted by l
    const int l = __builtin_ctz(tid | NT);
    const int cb = (n >> (l + 2)) + (tid >> (l + 1));
#pragma unroll
    for (int it = 0; it < FI; ++it) {
      const int t = (it * NT) / h, C = (it * NT) % h;
      if (t < Tact) {
        auto w = W + (t << LOGN);
        float2 lo, hi;
        io.fold(raw[it], tid + C, lo, hi);
        if (tid != 0) {
          const int cell = cb + (C >> (l + 1));
          w[cell] = lo;
          w[h + cell] = hi;
        } else if (C == 0) {
          w[0] = lo;  // c(0)
          w[h] = hi;  // c(N/2)
        } else {
          const int lc = __builtin_ctz(C);
          const int cell = (n >> (lc + 2)) + (C >> (lc + 1));
          w[cell] = lo;
          w[h + cell] = hi;
        }
      }
    }
  } else {
    constexpr int TS = NT / h;
    static_assert((TS * n) % kRowCells == 0, "fold rows step by whole row units");
    const int m = tid & (h - 1);
    const int t0 = tid >> (LOGN - 1);
    int c1 = 0, c2 = h;
    if (m != 0) {
      const int l = __builtin_ctz(m);
      c1 = (n >> (l + 2)) + (m >> (l + 1));
      c2 = h + c1;
    }
    const auto r1 = pad_row(W, (t0 << LOGN) + c1);
    const auto r2 = pad_row(W, (t0 << LOGN) + c2);
#pragma unroll
    for (int it = 0; it < FI; ++it) {
      if (t0 + it * TS < Tact) {
        float2 lo, hi;
        io.fold(raw[it], m, lo, hi);
        r1[it * TS * n] = lo;
        r2[it * TS * n] = hi;
      }
    }
  }
}

// Starts with a workgroup barrier (the fold's LDS stores); ends with the
// combine's LDS reads, unordered.
template <int LOGN, int T, int NT, int WAVE, bool SF = false, class Sync, class WSync,
          typename WP, class IO>
QFT_HD void tile_rest_s(const IO& io, WP W, int Tact, const float* sec, int tid, Sync sync,
                        WSync wsync) {
  constexpr int n = 1 << LOGN, h = n >> 1;
  constexpr int FI = tile_items<LOGN, T, NT>();
  const int tot_act = Tact << (LOGN - 1);
  sync();
  if constexpr (LOGN >= 3)
    sweeps_s<LOGN - 2, LOGN - 1, 2 * T, NT, WAVE, SIDES_ALT, true, SF>(W, sec, tid, sync,
                                                                       wsync);
  if constexpr (LOGN >= 5) {
    chain_fused<LOGN, T, NT, WAVE, true>(TileSides<WP>{W, LOGN}, io, Tact, tid, sync, wsync);
    return;
  }
  chain_s<LOGN, T, NT, WAVE>(W, tid, sync, wsync);
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int i = tid + it * NT;
    if (i < tot_act) {
      const int t = i >> (LOGN - 1);
      const int k = i & (h - 1);
      const auto Xt = io.out(t);
      auto w = W + (t << LOGN);
      if (k == 0) {
        io.put_edge(Xt, 0, w[0]);
        io.put_edge(Xt, h, w[h]);
      } else {
        io.put(Xt, n, k, w[k], w[h + k]);
      }
    }
  }
}

// SF as in fwd_chunk_s.
template <int LOGN, int T, int NT, int WAVE, bool SF = false, class Sync, class WSync,
          typename WP, class IO>
QFT_HD void tile_body_s(const IO& io, WP W, int Tact, const float* sec, int tid, Sync sync,
                        WSync wsync) {
  typename IO::Raw raw[tile_items<LOGN, T, NT>()];
  tile_fetch_s<LOGN, T, NT>(io, Tact, tid, raw);
  tile_fold_s<LOGN, T, NT>(io, W, Tact, tid, raw);
  tile_rest_s<LOGN, T, NT, WAVE, SF>(io, W, Tact, sec, tid, sync, wsync);
}

// Tile sources of tile_loop_s: how many tiles, a tile's descriptor, and from
// that the accessor and the transform count of the tile.
//  * a contiguous batch of `batch` transforms of 2^LOGN points, T per tile
//    (the last tile ragged); the descriptor is the tile index;
template <int DT, bool SWAP, int LOGN, int T>
struct ContigTiles {
  using IO = ContigIO<DT, SWAP, LOGN>;
  using Desc = int64_t;
  const typename Store<DT>::T* x;
  typename Store<DT>::T* X;
  int64_t batch;
  QFT_HD int64_t ntiles() const { return (batch + T - 1) / T; }
  QFT_HD Desc desc(int64_t w) const { return w; }
  QFT_HD IO io(Desc w) const { return IO(x + ((w * T) << LOGN), X + ((w * T) << LOGN)); }
  QFT_HD int count(Desc w) const { return (int)(batch - w * T < T ? batch - w * T : T); }
};
//  * the tile list of an uneven plan's group whose tiles each hold one
//    transform of 2^LOGN points: tile w = (log2n, first, 1, 0), the
//    transform at element offset offs[first].  Both lists are read-only for
//    the launch, so on the GPU they are read through the constant address
//    space: scalar loads, which do not wait behind the vector loads of the
//    next tile in flight (the offset is resolved once per tile, so the
//    combine's stores need no load either).
template <typename P>
QFT_HD P read_only(const P* p, int64_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(4))) P*)p)[i];
#else
  return p[i];
#endif
}
template <int DT, bool SWAP, int LOGN>
struct ListTiles {
  using IO = ContigIO<DT, SWAP, LOGN>;
  using Desc = int64_t;  // element offset of the tile's transform
  const typename Store<DT>::T* x;
  typename Store<DT>::T* X;
  const int4* tiles;
  const int64_t* offs;
  int64_t n;
  QFT_HD int64_t ntiles() const { return n; }
  QFT_HD Desc desc(int64_t w) const { return read_only(offs, (int64_t)read_only(tiles, w).y); }
  QFT_HD IO io(Desc o) const { return IO(x + o, X + o); }
  QFT_HD int count(Desc) const { return 1; }
};

// Persistent tiles: the workgroup takes tiles first, first + stride, .. <
// src.ntiles() and loads each next tile's x into registers while the
// current one runs its rounds in LDS, so that the loads overlap the LDS
// work.  The rounds must not read global memory (sec in LDS): the vector
// memory counter is in order, and a read issued after the loads would wait
// for them.  Before its first fold it calls pre() (the kernel's copy of the
// constant table into LDS, issued behind the first tile's loads).
template <int LOGN, int T, int NT, int WAVE, class Src, class Sync, class WSync, typename WP,
          class Pre>
QFT_HD void tile_loop_s(const Src& src, int64_t first, int64_t stride, WP W, const float* sec,
                        int tid, Sync sync, WSync wsync, Pre pre) {
  using IO = typename Src::IO;
  const int64_t ntiles = src.ntiles();
  if (first >= ntiles) return;
  typename IO::Raw raw[tile_items<LOGN, T, NT>()];
  typename Src::Desc d = src.desc(first);
  tile_fetch_s<LOGN, T, NT>(src.io(d), src.count(d), tid, raw);
  pre();
  for (int64_t w = first;;) {
    // per tile, so that the compiler does not hold every thread-dependent
    // LDS address of the bodies live across the loop
    launder(tid);
    const IO io = src.io(d);
    const int cnt = src.count(d);
    tile_fold_s<LOGN, T, NT>(io, W, cnt, tid, raw);
    const int64_t wn = w + stride;
    if (wn < ntiles) {
      d = src.desc(wn);
      tile_fetch_s<LOGN, T, NT>(src.io(d), src.count(d), tid, raw);
    }
    tile_rest_s<LOGN, T, NT, WAVE>(io, W, cnt, sec, tid, sync, wsync);
    if (wn >= ntiles) break;
    sync();  // the combine's LDS reads before the next fold's stores
    w = wn;
  }
}

// ===========================================================================
// Two-pass path for N = 8 MC, MC = 2^MC_LOG2 (one LDS segment = MC cells).
// A side has 4 MC cells: segment 0 is the head (blocks < MC, the DCT-0/DST-0
// chain up to P = 2 MC), segment 1 is the block of size MC, segments 2 and 3
// are the two halves of the block of size 2 MC (= N/4) after its top forward
// round.  Pass A: one workgroup per (transform, side, segment) gathers its
// cells straight from x (real fold of Sec. 4.2, and the top round for
// segments 2/3), runs the segment's remaining rounds in LDS and writes the
// heap buffer.  Pass B: streaming; the top backward round of block N/4, chain
// levels P = N/2 and N (eqs. qft_5C/5D/6) and the cdft combine (Sec. 4.1).
// ===========================================================================
// One side's DCT-0 (or DST-0) chain, levels P = 2 (4 for DST) .. 2^plog, on
// side cells sd[0 .. 2^(plog-1)) with the DCT top cell at *top.
template <bool DST, class Sync, class WSync, typename SP>
QFT_HD void chain_one_side(SP sd, SP top, int plog, int tid, int nthr, int wave_size, Sync sync,
                           WSync wsync) {
  constexpr int PW = 9;
  const int pw = plog < PW ? plog : PW;
  // small levels: wave 0 alone, ordered by wave-level syncs that every
  // thread executes (so that a full-barrier emulation stays uniform)
  const int lanes = nthr < wave_size ? nthr : wave_size;
  for (int p = DST ? 3 : 1; p <= pw; ++p) {
    if (tid < wave_size) {
      const int P = 1 << p;
      if (!DST && P == 2) {
        if (tid == 0) {
          const float2 a = sd[0], b = *top;
          sd[0] = cadd(a, b);
          *top = csub(a, b);
        }
      } else {
        const int ng = DST ? (P >> 3) : (P == 4 ? 1 : 1 + (P >> 3));
        for (int g = tid; g < ng; g += lanes) {
          if (DST) chain_dst_group(sd, P, g);
          else chain_dct_group(sd, top, P, g);
        }
      }
    }
    wsync();
  }
  sync();
  for (int p = (pw + 1 > (DST ? 3 : 1)) ? pw + 1 : (DST ? 3 : 1); p <= plog; ++p) {
    const int P = 1 << p;
    const int ng = DST ? (P >> 3) : 1 + (P >> 3);
    for (int g = tid; g < ng; g += nthr) {
      if (DST) chain_dst_group(sd, P, g);
      else chain_dct_group(sd, top, P, g);
    }
    sync();
  }
}

// Pass B, thread k of a transform (0 <= k < N/8).  Heap contents after pass A
// (DCT side; the DST side is alike with its own index conventions):
//   cells [0, MC) + top : D_{N/4} (chain output of the head)
//   cells [MC, 2MC)     : O1, the DCT-II of length N/8 (natural order)
//   cells [2MC, 3MC)    : A, cells [3MC, 4MC): T, the halves of the block N/4
// O0(2i) = A(i), O0(2i+1) = T(i) + T(i+1) (T(MC) = 0) is the top backward
// round of the block N/4; then chain levels N/2 and N and the combine.
template <int DT, bool SWAP, int MC_LOG2, typename GP>
QFT_HD void tp_pass_b(GP wt, typename Store<DT>::T* Xt, int k) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int N = 8 * MC, h = N / 2, q4 = N / 4, q8 = N / 8;
  auto dc = wt;
  auto ds = wt + h;
  // block N/4 outputs O0 (DCT, k' in [0, N/4)) and O0s (DST, k' in [1, N/4])
  auto O0 = [&](int kk) -> float2 {
    const int i = kk >> 1;
    if ((kk & 1) == 0) return dc[2 * MC + i];
    const float2 t0 = dc[3 * MC + i];
    return (i + 1 < MC) ? cadd(t0, (float2)dc[3 * MC + i + 1]) : t0;
  };
  auto O0s = [&](int kk) -> float2 {  // DST harmonic kk, stored at position kk-1
    const int pos = kk - 1, i = pos >> 1;
    if (pos & 1) return ds[2 * MC + i];
    const float2 t0 = ds[3 * MC + i];
    return (i >= 1) ? cadd((float2)ds[3 * MC + i - 1], t0) : t0;
  };
  auto put = [&](int kk, float2 C, float2 S) {  // X(kk), X(N-kk) from C(kk), S(kk)
    Store<DT>::st(Xt, kk, sw<SWAP>(make_float2(C.x + S.y, C.y - S.x)));
    Store<DT>::st(Xt, N - kk, sw<SWAP>(make_float2(C.x - S.y, C.y + S.x)));
  };
  if (k > 0) {
    // chain level N/2 at k and N/4 - k
    const float2 E = dc[k], o1 = dc[MC + k];
    const float2 a = cadd(E, o1), b = csub(E, o1);  // D_{N/2}(k), D_{N/2}(N/4-k)
    const float2 Es = ds[k], o1s = ds[MC + k - 1];
    const float2 as = cadd(o1s, Es), bs = csub(o1s, Es);  // S_{N/2}(k), S_{N/2}(N/4-k)
    // chain level N
    const float2 ok = O0(k), om = O0(q4 - k);
    const float2 oks = O0s(k), oms = O0s(q4 - k);
    put(k, cadd(a, ok), cadd(oks, as));
    put(h - k, csub(a, ok), csub(oks, as));
    put(q4 - k, cadd(b, om), cadd(oms, bs));
    put(q4 + k, csub(b, om), csub(oms, bs));
  } else {
    // DCT: D_{N/2}(0), D_{N/2}(N/4), D_{N/2}(N/8) = D_{N/4}(N/8) (top cell)
    const float2 E0 = dc[0], Et = dc[h], o10 = dc[MC];
    const float2 a0 = cadd(E0, o10), aq = csub(E0, o10);
    const float2 o0 = O0(0), o8 = O0(q8);
    const float2 C0 = cadd(a0, o0), Ch = csub(a0, o0);  // D_N(0), D_N(N/2)
    const float2 C4 = aq;                               // D_N(N/4) = D_{N/2}(N/4)
    const float2 C8 = cadd(Et, o8), C38 = csub(Et, o8); // D_N(N/8), D_N(3N/8)
    // DST: S_{N/2}(N/8) = O1s(N/8); S_N(N/8), S_N(3N/8); S_N(N/4) = O0s(N/4)
    const float2 s8 = ds[MC + q8 - 1];
    const float2 o8s = O0s(q8);
    const float2 S8 = cadd(o8s, s8), S38 = csub(o8s, s8);
    const float2 S4 = O0s(q4);
    Store<DT>::st(Xt, 0, sw<SWAP>(C0));
    Store<DT>::st(Xt, h, sw<SWAP>(Ch));
    put(q8, C8, S8);
    put(3 * q8, C38, S38);
    put(q4, C4, S4);
  }
}

// Pass A with both sides of one segment index j in the same workgroup: the
// DCT and DST cells of a position come from the same x samples (c = a + b,
// d = a - b), so x is gathered once for both.  LDS: DCT segment at L[0, MC),
// DST segment at L[MC, 2MC), the DCT top cell (c(N/2) / D(MC)) at L[2MC].
template <typename LP>
struct HeadSides {  // the head segments of pass A: DCT, DST and the top cell
  LP L;
  int mc;
  QFT_HD LP dc(int) const { return L; }
  QFT_HD LP ds(int) const { return L + mc; }
  QFT_HD LP top(int) const { return L + 2 * mc; }
};

// Segment j of a transform heap wt with sides of h cells once both sides'
// segment j is in LDS (DCT at L[0, MC), DST at L[MC, 2MC), for j = 0 the top
// cell at L[2MC]): the remaining rounds, for the head the DCT-0/DST-0 chain
// up to P = 2 MC, and the copy to the heap buffer.  Starts with a barrier
// (the caller's LDS stores) and leaves LDS being read.
template <int MC_LOG2, int NT, int WAVE, class Sync, class WSync, typename GP, typename LP>
QFT_HD void tp_segment(GP wt, LP L, int j, int h, const float* sec, int tid, Sync sync,
                       WSync wsync) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int NI = MC / NT;
  sync();
  if (j == 0) {
    sweeps_s<MC_LOG2 - 1, MC_LOG2, 2, NT, WAVE, SIDES_ALT, true>(L, sec, tid, sync, wsync);
    if constexpr (MC_LOG2 + 1 >= 5) {
      chain_fused<MC_LOG2 + 1, 1, NT, WAVE, false>(HeadSides<LP>{L, MC}, NoIO{}, 1, tid, sync,
                                                    wsync);
    } else {
      chain_one_side<false>(L, L + 2 * MC, MC_LOG2 + 1, tid, NT, WAVE, sync, wsync);
      chain_one_side<true>(L + MC, L + 2 * MC, MC_LOG2 + 1, tid, NT, WAVE, sync, wsync);
    }
  } else {
    sweeps_s<MC_LOG2, MC_LOG2, 2, NT, WAVE, SIDES_ALT, false>(L, sec, tid, sync, wsync);
  }
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int q = tid + it * NT;
    wt[j * MC + q] = (float2)L[q];
    if (!(j == 0 && q == 0)) wt[h + j * MC + q] = (float2)L[MC + q];
  }
  if (j == 0 && tid == 0) wt[h] = (float2)L[2 * MC];  // D_{2MC}(MC): top cell
}

// The x samples pass A needs for segment j of one transform, as stored
// (loaded by tp_load_a, folded into LDS by tp_fold_a):
//   j = 0: x(n), x(N - n), n = 4m for the thread's items m, and x(N/2)
//          (thread 0).  c(n), d(n) belong to heap cell M + (n >> (v + 1))
//          with v = ctz(n) and M = N >> (v + 2), the odd-time block of
//          periodization N / 2^v; item 0 is c(0) at cell 0 (it also loads
//          x(N - 4), unused).  Walking the head's cells in order would read
//          each block at its own stride (8 samples for the largest, up to
//          N/4); walking m reads x at a stride of 4 samples and scatters
//          into LDS instead;
//   j = 1: x(n), x(N - n), n = 4q + 2 (heap cell MC + q, the block N/8);
//   j >= 2: x(n), x(N - n), x(N/2 - n), x(N/2 + n), n = 2q + 1.
template <int DT, int NI>
struct TpRaw {
  using T = typename Store<DT>::T;
  T a[NI], b[NI], c[NI], d[NI];
  T top;
};

template <int DT, int MC_LOG2, int NT>
QFT_HD void tp_load_a(const typename Store<DT>::T* xt, int j, int tid,
                      TpRaw<DT, (1 << MC_LOG2) / NT>& r) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int N = 8 * MC, h = 4 * MC;
  constexpr int NI = MC / NT;
  if (j < 2) {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int q = tid + it * NT;
      const int n = j == 0 ? 4 * q : 4 * q + 2;
      r.a[it] = xt[n];
      r.b[it] = xt[N - (n == 0 ? 4 : n)];
    }
    if (j == 0 && tid == 0) r.top = xt[h];
  } else {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int n = 2 * (tid + it * NT) + 1;
      r.a[it] = xt[n];
      r.b[it] = xt[N - n];
      r.c[it] = xt[h - n];
      r.d[it] = xt[h + n];
    }
  }
}

// Fold (and for j >= 2 the top forward round) of the loaded samples into the
// LDS segments: DCT at L[0, MC), DST at L[MC, 2MC), the top cell at L[2MC].
template <int DT, bool SWAP, int MC_LOG2, int NT, typename LP>
QFT_HD void tp_fold_a(const TpRaw<DT, (1 << MC_LOG2) / NT>& r, int j, int tid,
                      const float* __restrict__ sec, LP L) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int N = 8 * MC;
  constexpr int NI = MC / NT;
  using S = Store<DT>;
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int q = tid + it * NT;
    const float2 a0 = sw<SWAP>(S::cvt(r.a[it])), b0 = sw<SWAP>(S::cvt(r.b[it]));
    float2 vc, vs;
    int cell = q;
    if (j == 0) {
      // head: n = 4q to heap cell M + (n >> (v + 1)), v = ctz(n), M = N >> (v + 2)
      const bool zero = q == 0;
      const int n = zero ? 4 : 4 * q;
      const int v = __builtin_ctz((unsigned)n);
      cell = zero ? 0 : (N >> (v + 2)) + (n >> (v + 1));
      vc = zero ? a0 : cadd(a0, b0);                  // c(0) for cell 0
      vs = zero ? make_float2(0.f, 0.f) : csub(a0, b0);
    } else if (j == 1) {
      vc = cadd(a0, b0);
      vs = csub(a0, b0);
    } else {
      // segments 2 and 3: the halves of the block N/4 after its top forward
      // round (S = 2 MC pairs odd n = 2q + 1 with N/2 - n)
      const float2 a1 = sw<SWAP>(S::cvt(r.c[it])), b1 = sw<SWAP>(S::cvt(r.d[it]));
      const float2 c0 = cadd(a0, b0), c1 = cadd(a1, b1);  // c(n), c(N/2-n)
      const float2 d0 = csub(a0, b0), d1 = csub(a1, b1);  // d(n), d(N/2-n)
      if (j == 2) {
        vc = cadd(c0, c1);
        vs = csub(d0, d1);
      } else {
        const float hs = sec[MC + q];
        vc = cscale(csub(c0, c1), hs);
        vs = cscale(cadd(d0, d1), hs);
      }
    }
    L[cell] = vc;
    L[MC + cell] = vs;
  }
  if (j == 0 && tid == 0) L[2 * MC] = sw<SWAP>(S::cvt(r.top));  // c(N/2)
}

// Pass A with both sides of one segment index j in the same workgroup: the
// DCT and DST cells of a position come from the same x samples (c = a + b,
// d = a - b), so x is gathered once for both.
template <int DT, bool SWAP, int MC_LOG2, int NT, int WAVE, class Sync, class WSync,
          typename GP, typename LP>
QFT_HD void tp_pass_a2(const typename Store<DT>::T* xt, GP wt, LP L, int j, const float* sec,
                       int tid, Sync sync, WSync wsync) {
  constexpr int MC = 1 << MC_LOG2;
  TpRaw<DT, MC / NT> r;
  tp_load_a<DT, MC_LOG2, NT>(xt, j, tid, r);
  tp_fold_a<DT, SWAP, MC_LOG2, NT>(r, j, tid, sec, L);
  tp_segment<MC_LOG2, NT, WAVE>(wt, L, j, 4 * MC, sec, tid, sync, wsync);
}

// Tile T of pass A: transform 8 (T / 32) + T % 8, segment (T / 8) % 4, so
// that the four workgroups of a transform share T % 8, i.e. the XCD under
// round-robin dispatch (and that XCD's L2 holds x for all four).
QFT_HD int64_t tp_tile_transform(int64_t T) { return (T >> 5) * 8 + (T & 7); }
QFT_HD int tp_tile_segment(int64_t T) { return (int)((T >> 3) & 3); }
// The first tile at or after T on the workgroup's stride whose transform is
// in the batch (the last group of eight transforms may be ragged).
QFT_HD int64_t tp_next_tile(int64_t T, int64_t stride, int64_t ntiles, int64_t batch) {
  while (T < ntiles && tp_tile_transform(T) >= batch) T += stride;
  return T;
}

// Pass-A threads per workgroup for N = 2^16 (2^13-cell segments, 32 cells
// each); N = 2^15 uses 256.
constexpr int kTpBlock13 = 512;

// Persistent pass A: the workgroup takes tiles first, first + stride, ..
// (tiles of transforms past the batch are skipped).  stride is a multiple of
// 32, so every tile of the workgroup has the same segment j, passed as a
// constant (each j gets its own code with only the registers it needs).
//
// Issuing the next tile's loads during the current tile's backward rounds
// and chain was measured and gained nothing: the gather is bound by the
// number of cache lines each workgroup requests (all of x, for every
// segment), not by their latency.
template <int J, int DT, bool SWAP, int MC_LOG2, int NT, int WAVE, class Sync, class WSync,
          typename GP, typename LP>
QFT_HD void tp_pass_a2_loop_j(const typename Store<DT>::T* x, GP W, LP L, int64_t batch,
                              int64_t ntiles, int64_t first, int64_t stride, const float* sec,
                              int tid, Sync sync, WSync wsync) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int logn = MC_LOG2 + 3;
  for (int64_t T = tp_next_tile(first, stride, ntiles, batch); T < ntiles;
       T = tp_next_tile(T + stride, stride, ntiles, batch)) {
    const int64_t t = tp_tile_transform(T);
    // Every LDS and table address of the body derives from tid; recomputing
    // them per tile keeps the compiler from holding hundreds of them live
    // across the loop (which spilled).
    launder(tid);
    TpRaw<DT, MC / NT> r;
    tp_load_a<DT, MC_LOG2, NT>(x + (t << logn), J, tid, r);
    tp_fold_a<DT, SWAP, MC_LOG2, NT>(r, J, tid, sec, L);
    tp_segment<MC_LOG2, NT, WAVE>(W + (t << logn), L, J, 4 * MC, sec, tid, sync, wsync);
    sync();  // the segment's last LDS reads before the next tile's LDS writes
  }
}

template <int DT, bool SWAP, int MC_LOG2, int NT, int WAVE, class Sync, class WSync,
          typename GP, typename LP>
QFT_HD void tp_pass_a2_loop(const typename Store<DT>::T* x, GP W, LP L, int64_t batch,
                            int64_t ntiles, int64_t first, int64_t stride, const float* sec,
                            int tid, Sync sync, WSync wsync) {
  switch (tp_tile_segment(first)) {
    case 0:
      tp_pass_a2_loop_j<0, DT, SWAP, MC_LOG2, NT, WAVE>(x, W, L, batch, ntiles, first, stride,
                                                        sec, tid, sync, wsync);
      break;
    case 1:
      tp_pass_a2_loop_j<1, DT, SWAP, MC_LOG2, NT, WAVE>(x, W, L, batch, ntiles, first, stride,
                                                        sec, tid, sync, wsync);
      break;
    case 2:
      tp_pass_a2_loop_j<2, DT, SWAP, MC_LOG2, NT, WAVE>(x, W, L, batch, ntiles, first, stride,
                                                        sec, tid, sync, wsync);
      break;
    default:
      tp_pass_a2_loop_j<3, DT, SWAP, MC_LOG2, NT, WAVE>(x, W, L, batch, ntiles, first, stride,
                                                        sec, tid, sync, wsync);
      break;
  }
}

// Segment pass of the multi-pass path: workgroup j of transform heap wt
// (sides of h cells) loads segment j of both sides (j = 0: the side heads
// and the top cell) and runs tp_segment on them.
template <int MC_LOG2, int NT, int WAVE, class Sync, class WSync, typename GP, typename LP>
QFT_HD void mp_segment_pair(GP wt, LP L, int h, int j, const float* sec, int tid, Sync sync,
                            WSync wsync) {
  constexpr int MC = 1 << MC_LOG2;
  constexpr int NI = MC / NT;
  float2 vc[NI], vs[NI];
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int q = tid + it * NT;
    vc[it] = wt[j * MC + q];
    vs[it] = wt[h + j * MC + q];
  }
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int q = tid + it * NT;
    L[q] = vc[it];
    L[MC + q] = vs[it];
  }
  if (j == 0 && tid == 0) L[2 * MC] = (float2)wt[h];  // top cell (DST cell 0)
  tp_segment<MC_LOG2, NT, WAVE>(wt, L, j, h, sec, tid, sync, wsync);
}

}  // namespace qftk
