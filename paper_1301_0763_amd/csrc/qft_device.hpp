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
  static QFT_HD float2 ld(const T* p, int64_t i) { return p[i]; }
  static QFT_HD void st(T* p, int64_t i, float2 v) { p[i] = v; }
};
template <> struct Store<1> {
  using T = __half2;
  static QFT_HD float2 ld(const T* p, int64_t i) { return __half22float2(p[i]); }
  static QFT_HD void st(T* p, int64_t i, float2 v) { p[i] = __float22half2_rn(v); }
};

template <bool SWAP> QFT_HD float2 sw(float2 v) {
  if constexpr (SWAP) return make_float2(v.y, v.x);
  else return v;
}

// ---------------------------------------------------------------------------
// Fold: x (T transforms of length n, global, element type DT) -> W (heap
// layout).  rdft fold of Sec. 4.2 and the cell map of the even/odd chain.
// ---------------------------------------------------------------------------
template <int DT, bool SWAP, typename WP>
QFT_HD void fold_to_heap(const typename Store<DT>::T* x, WP W, int logn, int T,
                          int tid, int nthr) {
  const int n = 1 << logn, h = n >> 1;
  const int total = T << (logn - 1);
  for (int i = tid; i < total; i += nthr) {
    const int t = i >> (logn - 1);
    const int m = i & (h - 1);
    const typename Store<DT>::T* xt = x + ((int64_t)t << logn);
    auto w = W + (t << logn);
    if (m == 0) {
      w[0] = sw<SWAP>(Store<DT>::ld(xt, 0));
      w[h] = sw<SWAP>(Store<DT>::ld(xt, h));
    } else {
      const float2 a = sw<SWAP>(Store<DT>::ld(xt, m));
      const float2 b = sw<SWAP>(Store<DT>::ld(xt, n - m));
      const int l = __builtin_ctz(m);
      const int cell = (n >> (l + 2)) + (m >> (l + 1));
      w[cell] = cadd(a, b);
      w[h + cell] = csub(a, b);
    }
  }
}

// ---------------------------------------------------------------------------
// Combine: heap layout W -> X (global), cdft combine of Sec. 4.1.
// ---------------------------------------------------------------------------
template <int DT, bool SWAP, typename WP>
QFT_HD void combine_from_heap(WP W, typename Store<DT>::T* X, int logn, int T,
                               int tid, int nthr) {
  const int n = 1 << logn, h = n >> 1;
  const int total = T << (logn - 1);
  for (int i = tid; i < total; i += nthr) {
    const int t = i >> (logn - 1);
    const int k = i & (h - 1);
    typename Store<DT>::T* Xt = X + ((int64_t)t << logn);
    auto w = W + (t << logn);
    if (k == 0) {
      Store<DT>::st(Xt, 0, sw<SWAP>(w[0]));
      Store<DT>::st(Xt, h, sw<SWAP>(w[h]));
    } else {
      const float2 C = w[k], S = w[h + k];
      Store<DT>::st(Xt, k, sw<SWAP>(make_float2(C.x + S.y, C.y - S.x)));
      Store<DT>::st(Xt, n - k, sw<SWAP>(make_float2(C.x - S.y, C.y + S.x)));
    }
  }
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

// G == 1 variant: K rounds 2^K, .., 2 on the whole segment j (S = 2^K).
template <int K, bool DST, typename SP>
QFT_HD void fwd_group_tail(SP sd, int j, const float* __restrict__ sec, bool skip0) {
  constexpr int S = 1 << K;
  const int base = j * S;
  float2 e[S];
#pragma unroll
  for (int c = 0; c < S; ++c) e[c] = sd[base + c];
#pragma unroll
  for (int m = K; m >= 1; --m) {
    const int span = 1 << m, half = span >> 1;
    float2 o[S];
#pragma unroll
    for (int i = 0; i < S; ++i) o[i] = e[i];
#pragma unroll
    for (int c0 = 0; c0 < S; c0 += span) {
      if (skip0 && j == 0 && c0 == 0) continue;
#pragma unroll
      for (int cc = 0; cc < half; ++cc) {
        const float2 a = e[c0 + cc], b = e[c0 + span - 1 - cc];
        const float hsec = sec[half + cc];
        const float2 s = cadd(a, b), d = csub(a, b);
        o[c0 + cc] = DST ? d : s;
        o[c0 + half + cc] = cscale(DST ? s : d, hsec);
      }
    }
#pragma unroll
    for (int i = 0; i < S; ++i) e[i] = o[i];
  }
#pragma unroll
  for (int c = 0; c < S; ++c) sd[base + c] = e[c];
}

// ---------------------------------------------------------------------------
// Backward round at segment size S on one item: output cells 2i, 2i+1 of
// segment j of one side.  Reads A(i), T(i) and the neighbour T(i+1) (DCT)
// or T(i-1) (DST).  Out of place: the caller stores after a barrier.
// ---------------------------------------------------------------------------
template <bool DST, typename SP>
QFT_HD void bwd_item(SP sd, int S, int j, int i, float2& y0, float2& y1) {
  const int hS = S >> 1;
  const int base = j * S;
  const float2 A = sd[base + i];
  const float2 T0 = sd[base + hS + i];
  if (!DST) {
    y0 = A;
    y1 = (i + 1 < hS) ? cadd(T0, sd[base + hS + i + 1]) : T0;
  } else {
    y1 = A;
    y0 = (i >= 1) ? cadd(sd[base + hS + i - 1], T0) : T0;
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


// ===========================================================================
// Sweeps over a workgroup's buffer.  A "side" is one half of a transform's
// heap (DCT or DST); transforms alternate DCT/DST sides, an isolated segment
// of a larger transform is a single side of fixed flavour.  Side s lives at
// W + s * 2^lgside.  `sync` is the workgroup barrier.
// ===========================================================================
enum SideMode { SIDES_ALT = 0, SIDES_DCT = 1, SIDES_DST = 2 };

QFT_HD bool side_is_dst(int mode, int s) {
  return mode == SIDES_ALT ? (s & 1) != 0 : mode == SIDES_DST;
}

// K forward rounds S = 2^hi .. 2^(hi-K+1).  TAIL: the rounds end at S = 2
// (G = 1, one group per segment); otherwise G = 2^(hi-K) >= 2.
template <int K, bool TAIL, typename WP>
QFT_HD void fwd_chunk(WP W, int lgside, int nsides, int mode, int hi, bool skip0,
                      const float* sec, int tid, int nthr) {
  const int lgGroups = TAIL ? (lgside - K) : (lgside - K - 1);  // groups per side
  const int total = nsides << lgGroups;
  for (int i = tid; i < total; i += nthr) {
    const int s = i >> lgGroups;
    const int g = i & ((1 << lgGroups) - 1);
    auto sd = W + (s << lgside);
    const bool dst = side_is_dst(mode, s);
    if (TAIL) {
      if (dst) fwd_group_tail<K, true>(sd, g, sec, skip0);
      else fwd_group_tail<K, false>(sd, g, sec, skip0);
    } else {
      const int lgHalfG = hi - K - 1;
      const int j = g >> lgHalfG;
      const int x = g & ((1 << lgHalfG) - 1);
      if (dst) fwd_group<K, true>(sd, 1 << hi, j, x, sec, skip0);
      else fwd_group<K, false>(sd, 1 << hi, j, x, sec, skip0);
    }
  }
}

// Forward rounds S = 2^top .. 2^bottom in chunks of <= 3 rounds aligned from
// the bottom; the chunk that ends at S = 2 uses the whole-segment form.
template <class Sync, typename WP>
QFT_HD void forward_sweep(WP W, int lgside, int nsides, int mode, int top, int bottom,
                          bool skip0, const float* sec, int tid, int nthr, Sync sync) {
  constexpr int KF = 3;
  if (top < bottom) return;
  const int R = top - bottom + 1;
  const int nchunks = (R + KF - 1) / KF;
  for (int c = nchunks - 1; c >= 0; --c) {
    const int lo = bottom + c * KF;
    const int hi = (top < lo + KF - 1) ? top : lo + KF - 1;
    const int K = hi - lo + 1;
    const bool tail = (lo == 1);
    if (K == 3) {
      if (tail) fwd_chunk<3, true>(W, lgside, nsides, mode, hi, skip0, sec, tid, nthr);
      else fwd_chunk<3, false>(W, lgside, nsides, mode, hi, skip0, sec, tid, nthr);
    } else if (K == 2) {
      if (tail) fwd_chunk<2, true>(W, lgside, nsides, mode, hi, skip0, sec, tid, nthr);
      else fwd_chunk<2, false>(W, lgside, nsides, mode, hi, skip0, sec, tid, nthr);
    } else {
      if (tail) fwd_chunk<1, true>(W, lgside, nsides, mode, hi, skip0, sec, tid, nthr);
      else fwd_chunk<1, false>(W, lgside, nsides, mode, hi, skip0, sec, tid, nthr);
    }
    sync();
  }
}

// Backward rounds S = 2^bottom .. 2^top, one round per pass: every thread
// loads its items into registers, the workgroup synchronises, then stores.
// Requires MAXI >= ceil(nsides * 2^(lgside-1) / nthr).
template <int MAXI, class Sync, typename WP>
QFT_HD void backward_sweep(WP W, int lgside, int nsides, int mode, int bottom, int top,
                           bool skip0, int tid, int nthr, Sync sync) {
  const int lgItems = lgside - 1;  // items (output cell pairs) per side
  const int total = nsides << lgItems;
  for (int s = bottom; s <= top; ++s) {
    const int S = 1 << s;
    float2 y0[MAXI], y1[MAXI];
#pragma unroll
    for (int it = 0; it < MAXI; ++it) {
      const int i = tid + it * nthr;
      if (i < total) {
        const int si = i >> lgItems;
        const int item = i & ((1 << lgItems) - 1);
        const int j = item >> (s - 1);
        const int ii = item & ((S >> 1) - 1);
        if (!(skip0 && j == 0)) {
          auto sd = W + (si << lgside);
          if (side_is_dst(mode, si)) bwd_item<true>(sd, S, j, ii, y0[it], y1[it]);
          else bwd_item<false>(sd, S, j, ii, y0[it], y1[it]);
        }
      }
    }
    sync();
#pragma unroll
    for (int it = 0; it < MAXI; ++it) {
      const int i = tid + it * nthr;
      if (i < total) {
        const int si = i >> lgItems;
        const int item = i & ((1 << lgItems) - 1);
        const int j = item >> (s - 1);
        const int ii = item & ((S >> 1) - 1);
        if (!(skip0 && j == 0)) {
          auto sd = W + (si << lgside);
          sd[j * S + 2 * ii] = y0[it];
          sd[j * S + 2 * ii + 1] = y1[it];
        }
      }
    }
    sync();
  }
}

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

template <class Sync, typename WP>
QFT_HD void chain_sweep(WP W, int logn, int T, int lo, int hi, int tid, int nthr, Sync sync) {
  for (int p = lo; p <= hi; ++p) {
    const int per_t = chain_groups(p);
    const int total = T * per_t;
    for (int i = tid; i < total; i += nthr) {
      const int t = i / per_t;
      const int g = i - t * per_t;
      chain_item(W + (t << logn), logn, p, g);
    }
    sync();
  }
}

// Everything between fold and combine for T transforms of 2^logn cells.
template <int MAXI, class Sync, typename WP>
QFT_HD void mid_sweeps(WP W, int logn, int T, const float* sec, int tid, int nthr, Sync sync) {
  if (logn >= 3) {
    forward_sweep(W, logn - 1, 2 * T, SIDES_ALT, logn - 2, 1, true, sec, tid, nthr, sync);
    backward_sweep<MAXI>(W, logn - 1, 2 * T, SIDES_ALT, 1, logn - 2, true, tid, nthr, sync);
  }
  chain_sweep(W, logn, T, 1, logn, tid, nthr, sync);
}

// ===========================================================================
// Whole-transform work of one workgroup: T transforms of length 2^logn.
// Transform t is read from x + off(t) and written to X + off(t), with
// off(t) = offs[t] when offs is given, else t * 2^logn.
// ===========================================================================
template <int DT, bool SWAP, int MAXI, class Sync, typename WP>
QFT_HD void tile_body(const typename Store<DT>::T* x, typename Store<DT>::T* X, WP W, int logn,
                      int T, const int64_t* offs, const float* sec, int tid, int nthr,
                      Sync sync) {
  const int n = 1 << logn, h = n >> 1;
  const int total = T << (logn - 1);
  for (int i = tid; i < total; i += nthr) {
    const int t = i >> (logn - 1);
    const int m = i & (h - 1);
    const int64_t o = offs ? offs[t] : ((int64_t)t << logn);
    const typename Store<DT>::T* xt = x + o;
    auto w = W + (t << logn);
    if (m == 0) {
      w[0] = sw<SWAP>(Store<DT>::ld(xt, 0));
      w[h] = sw<SWAP>(Store<DT>::ld(xt, h));
    } else {
      const float2 a = sw<SWAP>(Store<DT>::ld(xt, m));
      const float2 b = sw<SWAP>(Store<DT>::ld(xt, n - m));
      const int l = __builtin_ctz(m);
      const int cell = (n >> (l + 2)) + (m >> (l + 1));
      w[cell] = cadd(a, b);
      w[h + cell] = csub(a, b);
    }
  }
  sync();
  mid_sweeps<MAXI>(W, logn, T, sec, tid, nthr, sync);
  for (int i = tid; i < total; i += nthr) {
    const int t = i >> (logn - 1);
    const int k = i & (h - 1);
    const int64_t o = offs ? offs[t] : ((int64_t)t << logn);
    typename Store<DT>::T* Xt = X + o;
    auto w = W + (t << logn);
    if (k == 0) {
      Store<DT>::st(Xt, 0, sw<SWAP>(w[0]));
      Store<DT>::st(Xt, h, sw<SWAP>(w[h]));
    } else {
      const float2 C = w[k], S = w[h + k];
      Store<DT>::st(Xt, k, sw<SWAP>(make_float2(C.x + S.y, C.y - S.x)));
      Store<DT>::st(Xt, n - k, sw<SWAP>(make_float2(C.x - S.y, C.y + S.x)));
    }
  }
}

// ===========================================================================
// Multi-pass path (one transform too large for a workgroup).  Work items of
// the global passes over a heap buffer W of `batch` transforms.
// ===========================================================================
// fold item i < batch * N/2
template <int DT, bool SWAP, typename WP>
QFT_HD void mp_fold_item(const typename Store<DT>::T* x, WP W, int logn, int64_t i) {
  const int n = 1 << logn, h = n >> 1;
  const int64_t t = i >> (logn - 1);
  const int m = (int)(i & (h - 1));
  const typename Store<DT>::T* xt = x + (t << logn);
  auto w = W + (t << logn);
  if (m == 0) {
    w[0] = sw<SWAP>(Store<DT>::ld(xt, 0));
    w[h] = sw<SWAP>(Store<DT>::ld(xt, h));
  } else {
    const float2 a = sw<SWAP>(Store<DT>::ld(xt, m));
    const float2 b = sw<SWAP>(Store<DT>::ld(xt, n - m));
    const int l = __builtin_ctz(m);
    const int cell = (n >> (l + 2)) + (m >> (l + 1));
    w[cell] = cadd(a, b);
    w[h + cell] = csub(a, b);
  }
}

// combine item i < batch * N/2
template <int DT, bool SWAP, typename WP>
QFT_HD void mp_combine_item(WP W, typename Store<DT>::T* X, int logn, int64_t i) {
  const int n = 1 << logn, h = n >> 1;
  const int64_t t = i >> (logn - 1);
  const int k = (int)(i & (h - 1));
  typename Store<DT>::T* Xt = X + (t << logn);
  auto w = W + (t << logn);
  if (k == 0) {
    Store<DT>::st(Xt, 0, sw<SWAP>(w[0]));
    Store<DT>::st(Xt, h, sw<SWAP>(w[h]));
  } else {
    const float2 C = w[k], S = w[h + k];
    Store<DT>::st(Xt, k, sw<SWAP>(make_float2(C.x + S.y, C.y - S.x)));
    Store<DT>::st(Xt, n - k, sw<SWAP>(make_float2(C.x - S.y, C.y + S.x)));
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

// backward round S = 2^s, item i < 2*batch * N/4: Win -> Wout (cells [0, S)
// of each side, which are no block of this round, are copied unchanged).
template <typename RP, typename WP>
QFT_HD void mp_bwd_item(RP Win, WP Wout, int logn, int s, int64_t i) {
  const int lgside = logn - 1;
  const int lgItems = lgside - 1;
  const int S = 1 << s;
  const int64_t si = i >> lgItems;
  const int item = (int)(i & ((1 << lgItems) - 1));
  const int j = item >> (s - 1);
  const int ii = item & ((S >> 1) - 1);
  auto sin = Win + (si << lgside);
  auto sout = Wout + (si << lgside);
  if (j == 0) {
    sout[2 * ii] = sin[2 * ii];
    sout[2 * ii + 1] = sin[2 * ii + 1];
  } else {
    float2 y0, y1;
    if (si & 1) bwd_item<true>(sin, S, j, ii, y0, y1);
    else bwd_item<false>(sin, S, j, ii, y0, y1);
    sout[j * S + 2 * ii] = y0;
    sout[j * S + 2 * ii + 1] = y1;
  }
}

// chain level P = 2^p, item i < batch * chain_groups(p), in place.
template <typename WP>
QFT_HD void mp_chain_item(WP W, int logn, int p, int64_t i) {
  const int per_t = chain_groups(p);
  const int64_t t = i / per_t;
  const int g = (int)(i - t * per_t);
  chain_item(W + (t << logn), logn, p, g);
}

// Segment pass, one workgroup: block r of transform heap wt (length 2^logn)
// with segments of MC = 2^MC_LOG2 cells and LDS buffer L of 2 MC cells.
// r == 0: the core (both side heads [0, MC), a virtual transform of 2 MC
// cells; chain to P = 2 MC); r >= 1: segment j >= 1 of the DCT side, then of
// the DST side (rounds S = MC .. 2 and back; every sub-segment is a block).
template <int MC_LOG2, int MAXI, class Sync, typename GP, typename LP>
QFT_HD void mp_segment_body(GP wt, LP L, int logn, int r, const float* sec, int tid, int nthr,
                            Sync sync) {
  constexpr int MC = 1 << MC_LOG2;
  const int h = 1 << (logn - 1);
  const int segs = h >> MC_LOG2;
  if (r == 0) {
    for (int i = tid; i < 2 * MC; i += nthr) {
      const int side = i >> MC_LOG2, c = i & (MC - 1);
      L[i] = (float2)wt[side * h + c];
    }
    sync();
    mid_sweeps<MAXI>(L, MC_LOG2 + 1, 1, sec, tid, nthr, sync);
    for (int i = tid; i < 2 * MC; i += nthr) {
      const int side = i >> MC_LOG2, c = i & (MC - 1);
      wt[side * h + c] = (float2)L[i];
    }
  } else {
    const int side = (r - 1) / (segs - 1);
    const int j = 1 + (r - 1) - side * (segs - 1);
    auto seg = wt + (side * h + j * MC);
    for (int i = tid; i < MC; i += nthr) L[i] = (float2)seg[i];
    sync();
    const int mode = side ? SIDES_DST : SIDES_DCT;
    forward_sweep(L, MC_LOG2, 1, mode, MC_LOG2, 1, false, sec, tid, nthr, sync);
    backward_sweep<MAXI>(L, MC_LOG2, 1, mode, 1, MC_LOG2, false, tid, nthr, sync);
    for (int i = tid; i < MC; i += nthr) seg[i] = (float2)L[i];
  }
}

// Workgroups per transform of the segment pass.
QFT_HD int mp_segment_blocks(int logn, int mc_log2) {
  const int segs = 1 << (logn - 1 - mc_log2);
  return 1 + 2 * (segs - 1);
}

}  // namespace qftk
