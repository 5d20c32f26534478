// Fixed-point (integer) improved-QFT transform: the fixed-point use the
// paper recommends the method for (Sec. 1, Sec. 7), on gfx950.
//
// Number format: complex samples as int2 (real, imaginary), every addition
// and subtraction wrapping modulo 2^32; the only multiplications are the
// secant conversions of eq. qft_38A (and the two N = 8 base cases, which use
// the slice L = 1), with block-scaled constants: slice L (periodization 8L)
// holds mantissas H_L(m) = round(2^s_L / (2 cos(pi (2m+1) / (4L)))) < 2^30
// with one shift s_L per slice, and a product w * h is the 64-bit w H
// rounded half up at bit s_L, kept to 32 bits.  Every output is therefore a
// fixed function of the input integers: any order of the additions gives the
// same result, and the heap layout below computes exactly the values of the
// paper's recursion.
//
// Work layout: the heap layout of qft_device.hpp (sides of N/2 cells, the
// DCT-II / DST-II block of periodization P at cells [P/4, P/2) of its side,
// c(0) in cell 0, c(N/2) in cell N/2), one workgroup per transform (or a
// group of its threads), one round or chain level per pass:
//   fold             x -> c, d in heap order
//   forward rounds   S = N/4 .. 2, in place on closed quads of cells (two
//                    rounds per pass on closed groups of eight, fwd_round2,
//                    where the caller asks for it)
//   backward rounds  S = 2 .. N/4, from one buffer into the other, an item per
//                    pair of output cells
//   chain levels     P = 2 .. N, in place on closed groups
//   combine          X(k), X(N-k) from the DCT cell k and the DST cell k
// The buffers live in LDS (N <= 2^12) or in global scratch (2N cells per
// transform).  This path is written for exactness first: it takes one barrier
// per pass (a wavefront's ordering where one wavefront holds the transform).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#ifndef QFT_HD
#define QFT_HD __host__ __device__ __forceinline__
#endif

namespace qftk {
namespace fx {

QFT_HD int iadd(int a, int b) { return (int)((uint32_t)a + (uint32_t)b); }
QFT_HD int isub(int a, int b) { return (int)((uint32_t)a - (uint32_t)b); }
QFT_HD int2 add(int2 a, int2 b) { return make_int2(iadd(a.x, b.x), iadd(a.y, b.y)); }
QFT_HD int2 sub(int2 a, int2 b) { return make_int2(isub(a.x, b.x), isub(a.y, b.y)); }

// w * h with h = H / 2^s: the 64-bit product rounded half up at bit s, kept
// to the low 32 bits (two's complement).
QFT_HD int qmul(int w, int H, int s) {
  const int64_t p = (int64_t)w * (int64_t)H + ((int64_t)1 << (s - 1));
  return (int)(uint32_t)(uint64_t)(p >> s);
}
QFT_HD int2 mul(int2 w, int H, int s) { return make_int2(qmul(w.x, H, s), qmul(w.y, H, s)); }

// Constant table of the transform: H[L + m] (L = 1, 2, .., N/8, m < L) and
// the shift of slice L = 2^lg in shift[lg].
struct Table {
  const int* H;
  const int* shift;
};

// floor(log2 v), v >= 1
QFT_HD int ilog2(int v) { return 31 - __builtin_clz((unsigned)v); }

// Heap cell p >= 1 of a side holds the sample n = (2m + 1) N / (4M), M the
// largest power of two <= p, m = p - M.
QFT_HD int cell_sample(int p, int logn) {
  const int lgM = ilog2(p);
  return (2 * (p - (1 << lgM)) + 1) << (logn - 2 - lgM);
}

// Fold of x (Sec. 4.2: c(n) = x(n) + x(N-n), d(n) = x(n) - x(N-n)) into the
// heap: DCT side cells [0, N/2), DST side cells [N/2, N) (cell N/2 = c(N/2)).
template <typename XP, typename WP>
QFT_HD void fold(XP x, WP W, int logn, int tid, int nthr) {
  const int N = 1 << logn, h = N >> 1;
  for (int p = tid; p < h; p += nthr) {
    if (p == 0) {
      W[0] = x[0];
      W[h] = x[h];
    } else {
      const int n = cell_sample(p, logn);
      const int2 a = x[n], b = x[N - n];
      W[p] = add(a, b);
      W[h + p] = sub(a, b);
    }
  }
}

// Forward round S (Sec. 5.2.2-5.2.3, eqs. qft_1/qft_2, qft_38A) on every
// segment [jS, (j+1)S), j >= 1, of both sides: u(p) = y(p) + y(S-1-p),
// v(p) = y(p) - y(S-1-p) for p < S/2; DCT side u -> p, v h_{S/2}(p) -> S/2+p;
// DST side v -> p, u h_{S/2}(p) -> S/2+p.  Item = one closed quad of cells
// {p, S/2-1-p, S/2+p, S-1-p} (p < S/4; the pair {0, 1} when S = 2).
template <typename WP>
QFT_HD void fwd_round(WP W, int logn, int S, Table tab, int tid, int nthr) {
  const int h = 1 << (logn - 1);
  const int L = S >> 1;
  const int lgS = ilog2(S);
  const int s = tab.shift[lgS - 1];
  const int* H = tab.H + L;
  const int lgq = S >= 4 ? lgS - 2 : 0;     // quads per segment: 2^lgq
  const int per_side = ((h >> lgS) - 1) << lgq;  // segments j = 1 .. h/S - 1
  const int items = 2 * per_side;
  for (int i = tid; i < items; i += nthr) {
    const int side = i >= per_side ? 1 : 0;
    const int r = i - side * per_side;
    const int j = 1 + (r >> lgq), p = r & ((1 << lgq) - 1);
    auto y = W + side * h + j * S;
    const bool dst = side != 0;
    if (S == 2) {
      const int2 a = y[0], b = y[1];
      const int2 u = add(a, b), v = sub(a, b);
      y[0] = dst ? v : u;
      y[1] = mul(dst ? u : v, H[0], s);
    } else {
      const int pa = p, pb = L - 1 - p, pc = L + p, pd = S - 1 - p;
      const int2 a = y[pa], b = y[pb], c = y[pc], d = y[pd];
      const int2 u1 = add(a, d), v1 = sub(a, d);  // pair (p, S-1-p)
      const int2 u2 = add(b, c), v2 = sub(b, c);  // pair (L-1-p, L+p)
      y[pa] = dst ? v1 : u1;
      y[pc] = mul(dst ? u1 : v1, H[pa], s);
      y[pb] = dst ? v2 : u2;
      y[pd] = mul(dst ? u2 : v2, H[pb], s);
    }
  }
}

// One forward quad in registers: the pairs (a, d) and (b, c) of a round's
// closed quad {pa, pb, pc, pd} (values a, b, c, d), outputs in the same cells,
// with the slice's constants H(pa), H(pb) and shift s (as in fwd_round).
QFT_HD void fwd_quad(int2& a, int2& b, int2& c, int2& d, int ha, int hb, int s, bool dst) {
  const int2 u1 = add(a, d), v1 = sub(a, d);
  const int2 u2 = add(b, c), v2 = sub(b, c);
  a = dst ? v1 : u1;
  c = mul(dst ? u1 : v1, ha, s);
  b = dst ? v2 : u2;
  d = mul(dst ? u2 : v2, hb, s);
}

// Forward rounds S and S/2 (S >= 8) in one pass, the same operations as two
// fwd_round passes.  With L = S/2 and M = S/4, round S's quads p and M-1-p
// (p < S/8) of a segment j >= 1 hold the eight cells {p, M-1-p, M+p, L-1-p,
// L+p, L+M-1-p, L+M+p, S-1-p}, which after that round are round S/2's quad p
// of the segment's lower half and of its upper half: a closed group of eight.
// Round S skips the head segment (j = 0), round S/2 only the lower half of it,
// so the head's items are round S/2's quads of [L, S) alone.
template <typename WP>
QFT_HD void fwd_round2(WP W, int logn, int S, Table tab, int tid, int nthr) {
  const int h = 1 << (logn - 1);
  const int L = S >> 1, M = S >> 2;
  const int lgS = ilog2(S);
  const int s1 = tab.shift[lgS - 1], s2 = tab.shift[lgS - 2];
  const int* H1 = tab.H + L;  // round S: slice L
  const int* H2 = tab.H + M;  // round S/2: slice L/2
  const int lgg = lgS - 3;    // groups per segment: S/8
  const int per_side = (h >> lgS) << lgg;
  for (int i = tid; i < 2 * per_side; i += nthr) {
    const int side = i >= per_side ? 1 : 0;
    const int r = i - side * per_side;
    const int j = r >> lgg, p = r & ((1 << lgg) - 1);
    auto y = W + side * h + j * S;
    const bool dst = side != 0;
    const int q = M - 1 - p;
    if (j == 0) {
      auto z = y + L;
      int2 a = z[p], b = z[q], c = z[M + p], d = z[L - 1 - p];
      fwd_quad(a, b, c, d, H2[p], H2[q], s2, dst);
      z[p] = a;
      z[q] = b;
      z[M + p] = c;
      z[L - 1 - p] = d;
      continue;
    }
    int2 c0 = y[p], c1 = y[q], c2 = y[M + p], c3 = y[L - 1 - p];
    int2 c4 = y[L + p], c5 = y[L + q], c6 = y[L + M + p], c7 = y[S - 1 - p];
    // round S: quad p = {p, L-1-p, L+p, S-1-p}, quad q = {q, L-1-q, L+q, S-1-q}
    // (L-1-q = M+p, S-1-q = L+M+p)
    fwd_quad(c0, c3, c4, c7, H1[p], H1[L - 1 - p], s1, dst);
    fwd_quad(c1, c2, c5, c6, H1[q], H1[M + p], s1, dst);
    // round S/2: quad p of [0, L) = {p, q, M+p, L-1-p}, of [L, S) likewise
    fwd_quad(c0, c1, c2, c3, H2[p], H2[q], s2, dst);
    fwd_quad(c4, c5, c6, c7, H2[p], H2[q], s2, dst);
    y[p] = c0;
    y[q] = c1;
    y[M + p] = c2;
    y[L - 1 - p] = c3;
    y[L + p] = c4;
    y[L + q] = c5;
    y[L + M + p] = c6;
    y[S - 1 - p] = c7;
  }
}

// Backward round S (eq. qft_4B interleave, eqs. qft_38B corrected / qft_38C,
// the dst_oo special case) from Win into Wout: for every segment j >= 1 with
// halves A = [jS, jS + S/2) and T = [jS + S/2, (j+1)S):
//   DCT: Y(2i) = A(i), Y(2i+1) = T(i) + T(i+1), T(S/2) = 0;
//   DST: Y(2i+1) = A(i), Y(2i) = T(i-1) + T(i), T(-1) = 0;
// the head cells [0, S) of each side are carried over unchanged.
template <typename RP, typename WP>
QFT_HD void bwd_round(RP Win, WP Wout, int logn, int S, int tid, int nthr) {
  const int h = 1 << (logn - 1);
  const int L = S >> 1;
  const int lgS = ilog2(S);
  const int hp = h >> 1;  // output pairs (cells 2i, 2i+1) per side
  // item: one pair of output cells, so that every lane of a wavefront takes
  // the same branch of its side (rounds exist for N >= 8, so h >= 4)
  for (int c = tid; c < 2 * hp; c += nthr) {
    const int side = c >= hp ? 1 : 0;
    const int q = 2 * (c - side * hp);
    auto in = Win + side * h;
    auto out = Wout + side * h;
    if (q < S) {
      out[q] = in[q];
      out[q + 1] = in[q + 1];
      continue;
    }
    const int j = q >> lgS, i = (q & (S - 1)) >> 1;
    auto a = in + j * S;
    auto t = a + L;
    int2 ye, yo;
    if (side == 0) {
      ye = a[i];
      yo = (i + 1 < L) ? add(t[i], t[i + 1]) : (int2)t[i];
    } else {
      yo = a[i];
      ye = (i >= 1) ? add(t[i - 1], t[i]) : (int2)t[i];
    }
    out[q] = ye;
    out[q + 1] = yo;
  }
}

// Chain level P (eqs. qft_5C, qft_5D, qft_6), both sides, in place.
//   DCT (P >= 4): E = D_{P/2} in cells [0, P/4) and E(P/4) in the top cell
//     N/2, O(k) in cell P/4 + k; D(k) = E(k) + O(k), D(P/2-k) = E(k) - O(k)
//     (k < P/4), D(P/4) = E(P/4); D(k) -> cell k, D(P/2) -> top cell.
//     P = 2: D(0) = c(0) + c(N/2) -> cell 0, D(1) = c(0) - c(N/2) -> top.
//     Groups: k = 0 (cells 0, P/4, top), k with P/4 - k (1 <= k < P/8), P/8.
//   DST (P >= 8): E(k) in cell k (1 <= k < P/4), O(k) in cell P/4 + k - 1
//     (1 <= k <= P/4); S(k) = O(k) + E(k), S(P/2-k) = O(k) - E(k), S(P/4) =
//     O(P/4); S(k) -> cell k.  Groups: k = 1 with O(P/4), k with P/4 + 1 - k
//     (2 <= k <= P/8).
template <typename WP>
QFT_HD void chain_level(WP W, int logn, int P, int tid, int nthr) {
  const int h = 1 << (logn - 1);
  auto dc = W;
  auto ds = W + h;
  auto top = W + h;  // DST cell 0 holds the DCT's top value
  const int q = P >> 2;
  const int dct_items = P == 2 ? 1 : 1 + (P >= 8 ? P / 8 : 0);
  const int dst_items = P >= 8 ? P / 8 : 0;
  for (int i = tid; i < dct_items + dst_items; i += nthr) {
    if (i < dct_items) {
      if (P == 2) {
        const int2 e = dc[0], t = top[0];
        dc[0] = add(e, t);
        top[0] = sub(e, t);
      } else if (i == 0) {
        const int2 e0 = dc[0], o0 = dc[q], eq = top[0];
        dc[0] = add(e0, o0);
        top[0] = sub(e0, o0);
        dc[q] = eq;
      } else {
        const int k = i, kp = q - k;  // k = P/8 pairs with itself
        const int2 ek = dc[k], ok = dc[q + k];
        if (kp != k) {
          const int2 ep = dc[kp], op = dc[q + kp];
          dc[kp] = add(ep, op);
          dc[(P >> 1) - kp] = sub(ep, op);
        }
        dc[k] = add(ek, ok);
        dc[(P >> 1) - k] = sub(ek, ok);
      }
    } else {
      const int k = 1 + (i - dct_items);  // 1 .. P/8
      if (k == 1) {
        const int2 e1 = ds[1], o1 = ds[q], oq = ds[(P >> 1) - 1];
        ds[1] = add(o1, e1);
        ds[(P >> 1) - 1] = sub(o1, e1);
        ds[q] = oq;
      } else {
        const int kp = q + 1 - k;
        const int2 ek = ds[k], ok = ds[q + k - 1];
        const int2 ep = ds[kp], op = ds[q + kp - 1];
        ds[k] = add(ok, ek);
        ds[(P >> 1) - k] = sub(ok, ek);
        ds[kp] = add(op, ep);
        ds[(P >> 1) - kp] = sub(op, ep);
      }
    }
  }
}

// Combine (Sec. 4.1): with C = DCT cell k = (Cr, Ci) and S = DST cell k =
// (Sr, Si), X(k) = (Cr + Si, Ci - Sr), X(N-k) = (Cr - Si, Ci + Sr) for
// 0 < k < N/2; X(0) = C(0), X(N/2) = the top cell.
template <typename WP, typename XP>
QFT_HD void combine(WP W, XP X, int logn, int tid, int nthr) {
  const int N = 1 << logn, h = N >> 1;
  for (int k = tid; k <= h; k += nthr) {
    if (k == 0) {
      X[0] = W[0];
    } else if (k == h) {
      X[h] = W[h];
    } else {
      const int2 c = W[k], s = W[h + k];
      X[k] = make_int2(iadd(c.x, s.y), isub(c.y, s.x));
      X[N - k] = make_int2(isub(c.x, s.y), iadd(c.y, s.x));
    }
  }
}

// Host: the integer constant table for transforms up to 2^log2n_max points
// (N/4 mantissas, layout of the FP32 table: entry L + m), shift[lg] for the
// slice L = 2^lg.  h_L(m) = 1/(2 cos(pi (2m+1) / (4L))) in FP64 (C library
// cosine), e_L the binary exponent of h_L(L-1) (h < 2^e_L), s_L = 30 - e_L,
// H_L(m) = floor(h_L(m) 2^s_L + 1/2).  Entry 0 is unused (0).
inline void fill_table_q(int* H, int* shift, int log2n_max) {
  const int64_t nt = ((int64_t)1 << (log2n_max < 3 ? 3 : log2n_max)) / 4;
  H[0] = 0;
  int lg = 0;
  for (int64_t L = 1; 2 * L <= nt; L *= 2, ++lg) {
    double hmax = 0.0;
    for (int64_t m = 0; m < L; ++m) {
      const double hv = 1.0 / (2.0 * std::cos(M_PI * (double)(2 * m + 1) / (double)(4 * L)));
      if (m == L - 1) hmax = hv;
    }
    int e = 0;
    (void)std::frexp(hmax, &e);
    const int sh = 30 - e;
    shift[lg] = sh;
    for (int64_t m = 0; m < L; ++m) {
      const double hv = 1.0 / (2.0 * std::cos(M_PI * (double)(2 * m + 1) / (double)(4 * L)));
      H[L + m] = (int)std::floor(hv * std::ldexp(1.0, sh) + 0.5);
    }
  }
}

// One transform of 2^logn points, x -> X, with heap buffers B0, B1 of N
// cells each; every pass ends with sync() (a workgroup barrier, or the
// wavefront's own ordering where one wavefront holds the transform's threads).
// fuse2: forward rounds two per pass (fwd_round2) down to S = 8, which halves
// those passes but also the items per pass.
template <typename XP, typename OP, typename BP, class Sync>
QFT_HD void transform(XP x, OP X, BP B0, BP B1, int logn, Table tab, int tid, int nthr,
                      Sync sync, bool fuse2) {
  fold(x, B0, logn, tid, nthr);
  sync();
  int S = (1 << logn) >> 2;
  for (; fuse2 && S >= 8; S >>= 2) {
    fwd_round2(B0, logn, S, tab, tid, nthr);
    sync();
  }
  for (; S >= 2; S >>= 1) {
    fwd_round(B0, logn, S, tab, tid, nthr);
    sync();
  }
  BP cur = B0, oth = B1;
  for (int S = 2; S <= ((1 << logn) >> 2); S <<= 1) {
    bwd_round(cur, oth, logn, S, tid, nthr);
    sync();
    BP t = cur;
    cur = oth;
    oth = t;
  }
  for (int P = 2; P <= (1 << logn); P <<= 1) {
    chain_level(cur, logn, P, tid, nthr);
    sync();
  }
  combine(cur, X, logn, tid, nthr);
}

}  // namespace fx
}  // namespace qftk
