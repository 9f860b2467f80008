// Stockham autosort FFT core for power-of-two lengths, radix 8/4/2.
//
// A line of length L is owned by TPL = L/R threads; thread t holds the R
// elements at positions t + s*TPL (s = 0..R-1) in registers.  Each stage
// reads its butterflies' inputs from those registers, applies the stage
// twiddles, does a radix-r DFT in registers and scatters the outputs to LDS
// in Stockham order; after a barrier every thread re-reads positions
// t + s*TPL, which are exactly the inputs of its next-stage butterflies (r
// always divides R).
//
// Stage order: the one stage whose radix is smaller than R (when log2 L is
// not a multiple of log2 R) comes first, every later stage has radix R.  The
// last stage then has one butterfly per thread whose outputs are positions
// t + s*TPL of the natural-order result, so it stays in registers and the
// transform makes (stages - 1) trips through LDS.
//
// Lines of stride 1 (one line per thread group, as in the row transform)
// pad their LDS image by one slot every 8 elements: element p sits at slot
// p + p/8.  Without the pad the radix-r scatter of the first stage puts the
// lanes of a wave r elements apart, which maps them to the same banks.
// Strided lines (several adjacent columns per workgroup) already give each
// 8-lane group a contiguous run and are not padded.
//
// Twiddles: each stage after the first needs w^s, s = 1..R-1, with
// w = e^{-+2 pi i k/(NS R)} for its butterfly index k.  Only w is read from
// the table, before the barrier that precedes the stage, so the load
// overlaps the wait; the powers are formed by products (a few ulp, within
// the transform's own O(log L) rounding).
//
// Sign convention: SIGN = -1 computes X_k = sum_j x_j e^{-2 pi i jk/L}
// (forward), SIGN = +1 the same sum with e^{+...} (unnormalised inverse).
// Twiddles come from a table tw[j] = exp(-2 pi i j / TW_N), TW_N = 2^TW_LOG,
// generated on the host in extended precision.
#pragma once
#include "cx.hpp"

namespace expdiag {

constexpr int TW_LOG = 12;
constexpr int TW_N = 1 << TW_LOG;

template <int S, typename T>
__device__ __forceinline__ void bf2(cx<T>* a) {
  cx<T> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}

template <int S, typename T>
__device__ __forceinline__ void bf4(cx<T>& a0, cx<T>& a1, cx<T>& a2,
                                    cx<T>& a3) {
  cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3;
  cx<T> t3 = mul_si<S>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <int S, typename T>
__device__ __forceinline__ void bf8(cx<T>* a) {
  // even / odd halves
  cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  bf4<S>(e0, e1, e2, e3);
  bf4<S>(o0, o1, o2, o3);
  const T h = static_cast<T>(0.70710678118654752440084436210484904);
  // o1 *= (1 + S i)/sqrt2 ; o2 *= S i ; o3 *= (-1 + S i)/sqrt2
  o1 = mk<T>(h * (o1.x - S * o1.y), h * (S * o1.x + o1.y));
  o2 = mul_si<S>(o2);
  o3 = mk<T>(h * (-o3.x - S * o3.y), h * (S * o3.x - o3.y));
  a[0] = e0 + o0;
  a[4] = e0 - o0;
  a[1] = e1 + o1;
  a[5] = e1 - o1;
  a[2] = e2 + o2;
  a[6] = e2 - o2;
  a[3] = e3 + o3;
  a[7] = e3 - o3;
}

template <int r, int S, typename T>
__device__ __forceinline__ void butterfly(cx<T>* a) {
  if constexpr (r == 2)
    bf2<S>(a);
  else if constexpr (r == 4)
    bf4<S>(a[0], a[1], a[2], a[3]);
  else
    bf8<S>(a);
}

template <int S, typename T>
__device__ __forceinline__ cx<T> twid(const cx<T>* tw, int j) {
  cx<T> w = gld(tw, j);
  if constexpr (S > 0) w.y = -w.y;
  return w;
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// Elements per thread for a line of length L (at most RMAX).
template <int L, int RMAX = 8>
struct FftShape {
  static constexpr int R = L >= RMAX ? RMAX : L;
  static constexpr int TPL = L / R;
};

// Barrier among the threads that share a line's LDS data: the whole block,
// or, when every line lives inside one wavefront (WAVE), just that
// wavefront.  A wavefront's lanes execute together and its LDS operations
// complete in issue order, so there a compiler-level fence is all that is
// needed and the block's other wavefronts run on independently.
template <bool WAVE>
__device__ __forceinline__ void line_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// LDS slot of element p of a line (padded for stride-1 lines).
template <bool PAD>
__device__ __forceinline__ int slot(int p) {
  return PAD ? p + (p >> 3) : p;
}
// Slots one line of n elements occupies.
constexpr int line_slots(int n, bool pad) {
  return pad ? n + ((n - 1) >> 3) : n;
}

// Radix of the stage with span NS: the remainder radix first, then R.
template <int L, int R, int NS>
constexpr int stage_radix() {
  constexpr int rb = R > 1 ? ilog2c(L / NS) % ilog2c(R) : 0;
  return rb == 0 ? R : (1 << rb);
}

// a[s] *= w^s, s = 1..r-1
template <int r, typename T>
__device__ __forceinline__ void apply_twiddles(cx<T>* a, cx<T> w1) {
  if constexpr (r >= 2) a[1] = cmul(a[1], w1);
  if constexpr (r >= 4) {
    const cx<T> w2 = cmul(w1, w1);
    const cx<T> w3 = cmul(w2, w1);
    a[2] = cmul(a[2], w2);
    a[3] = cmul(a[3], w3);
    if constexpr (r == 8) {
      const cx<T> w4 = cmul(w2, w2);
      a[4] = cmul(a[4], w4);
      a[5] = cmul(a[5], cmul(w4, w1));
      a[6] = cmul(a[6], cmul(w4, w2));
      a[7] = cmul(a[7], cmul(w4, w3));
    }
  }
}

// One Stockham stage with span NS, then recurse.  `lds` points at element 0
// of this thread's line; element p lives at lds[slot<PAD>(p) * stride].
// w1 is this stage's base twiddle (unused when NS == 1).  OUT_LDS: also
// leave the natural-order result in LDS (a barrier follows before anyone
// reads it).  PPOFF > 0: two LDS images PPOFF elements apart, exchanges
// alternating between them starting with image BUF; an exchange then
// needs only the barrier between its writes and reads, because the next
// exchange writes the other image and the one after waits behind that
// exchange's barrier, which every thread reaches only after its reads.
template <typename T, int L, int R, int S, int NS, bool PAD, bool OUT_LDS,
          bool WAVE, int ST = 0, bool PRE = false, int PPOFF = 0, int BUF = 0>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[R], cx<T> w1,
                                           cx<T>* lds, int stride, int t,
                                           const cx<T>* tw) {
  constexpr int TPL = L / R;
  constexpr int r = stage_radix<L, R, NS>();
  constexpr int NB = R / r;
  static_assert(NS == 1 || NB == 1, "only the first stage has a small radix");
  if constexpr (NS * r == L) {
    // last stage: one butterfly per thread, outputs t + s*TPL
    static_assert(NB == 1, "last stage has radix R");
    cx<T> a[R];
#pragma unroll
    for (int s = 0; s < R; ++s) a[s] = v[s];
    if constexpr (NS > 1) apply_twiddles<R>(a, w1);
    butterfly<R, S>(a);
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = a[s];
    if constexpr (OUT_LDS) {
#pragma unroll
      for (int s = 0; s < R; ++s)
        lds[slot<PAD>(t + s * TPL) * stride] = v[s];
    }
  } else {
    cx<T>* img = lds + BUF * PPOFF;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int b = t + q * TPL;
      const int k = b & (NS - 1);
      cx<T> a[r];
#pragma unroll
      for (int s = 0; s < r; ++s) a[s] = v[q + s * NB];
      if constexpr (NS > 1) apply_twiddles<r>(a, w1);
      butterfly<r, S>(a);
      const int base = (b / NS) * NS * r + k;
#pragma unroll
      for (int s = 0; s < r; ++s)
        img[slot<PAD>(base + s * NS) * stride] = a[s];
    }
    // next stage: span NS*r, radix R, one butterfly (index t) per thread;
    // PRE: `tw` holds the stages' base twiddles (forward sign), already in
    // registers (fft_stage_twiddles)
    constexpr int NS2 = NS * r;
    constexpr int sh2 = TW_LOG - ilog2c(NS2 * R);
    cx<T> w2;
    if constexpr (PRE)
      w2 = S > 0 ? conj(tw[ST + 1]) : tw[ST + 1];
    else
      w2 = twid<S>(tw, (t & (NS2 - 1)) << sh2);
    line_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = img[slot<PAD>(t + s * TPL) * stride];
    if constexpr ((NS2 * R < L && PPOFF == 0) || OUT_LDS) line_sync<WAVE>();
    fft_stages<T, L, R, S, NS2, PAD, OUT_LDS, WAVE, ST + 1, PRE, PPOFF,
               (PPOFF > 0 ? 1 - BUF : 0)>(v, w2, lds, stride, t, tw);
  }
}

// e^{-i pi j / 8}, j = 0..7 (exact to the last bit in fp64)
template <typename T>
__device__ __forceinline__ cx<T> eighth_root(int j) {
  constexpr long double C1 = 0.92387953251128675612818318939678829L;
  constexpr long double S1 = 0.38268343236508977172845998403039887L;
  constexpr long double H = 0.70710678118654752440084436210484904L;
  const long double re[8] = {1.0L, C1, H, S1, 0.0L, -S1, -H, -C1};
  const long double im[8] = {0.0L, -S1, -H, -C1, -1.0L, -C1, -H, -S1};
  return mk<T>(static_cast<T>(re[j]), static_cast<T>(im[j]));
}

// Number of stages of a length-L transform with R elements per thread.
template <int L, int R, int NS = 1>
constexpr int fft_stage_count() {
  if constexpr (NS >= L) {
    return 0;
  } else {
    return 1 + fft_stage_count<L, R, NS * stage_radix<L, R, NS>()>();
  }
}

// Base twiddle (forward sign) of every stage after the first for thread t:
// w[st] for stage st = 1 .. stages-1 (w[0] unused).  Lets a caller issue
// these loads together with its data loads (fft_line_pre).
template <typename T, int L, int R, int NS = 1, int ST = 0>
__device__ __forceinline__ void fft_stage_twiddles(cx<T>* w, int t,
                                                   const cx<T>* tw) {
  if constexpr (NS * stage_radix<L, R, NS>() < L) {
    constexpr int NS2 = NS * stage_radix<L, R, NS>();
    constexpr int sh2 = TW_LOG - ilog2c(NS2 * R);
    w[ST + 1] = gld(tw, (t & (NS2 - 1)) << sh2);
    fft_stage_twiddles<T, L, R, NS2, ST + 1>(w, t, tw);
  }
}

// Full FFT of one line.  Precondition: v[s] holds element t + s*TPL and no
// thread still reads this line's LDS (callers place a barrier before).
// Postcondition: natural-order result in v (positions t + s*TPL) and, with
// OUT_LDS, in LDS as well (visible after the caller's next barrier).
// Every thread of the block (WAVE: of the wavefront) must call this (it
// contains barriers).
template <typename T, int L, int S, bool PAD = false, bool OUT_LDS = false,
          bool WAVE = false, int R>
__device__ __forceinline__ void fft_line(cx<T> (&v)[R], cx<T>* lds,
                                         int stride, int t, const cx<T>* tw) {
  if constexpr (L == 1) {
    if constexpr (OUT_LDS) lds[0] = v[0];
    return;
  } else {
    fft_stages<T, L, R, S, 1, PAD, OUT_LDS, WAVE>(v, mk<T>(1, 0), lds, stride,
                                                  t, tw);
  }
}

// fft_line with the stage twiddles already loaded (fft_stage_twiddles).
// PPOFF > 0: exchanges alternate between two LDS images PPOFF elements
// apart, the first in image BUF (fft_stages); the transform makes
// fft_exchanges<L, R>() of them, so a following transform that starts in
// the other image than the last one written needs no barrier before it.
template <typename T, int L, int S, int R, int PPOFF = 0, int BUF = 0>
__device__ __forceinline__ void fft_line_pre(cx<T> (&v)[R], cx<T>* lds,
                                             int stride, int t,
                                             const cx<T>* wst) {
  if constexpr (L > 1)
    fft_stages<T, L, R, S, 1, false, false, false, 0, true, PPOFF, BUF>(
        v, mk<T>(1, 0), lds, stride, t, wst);
}

// Trips through LDS of a length-L transform with R elements per thread.
template <int L, int R>
constexpr int fft_exchanges() {
  return L > 1 ? fft_stage_count<L, R>() - 1 : 0;
}

}  // namespace expdiag
