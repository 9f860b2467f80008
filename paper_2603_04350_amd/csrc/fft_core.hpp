// Stockham autosort FFT core for power-of-two lengths, radix 8/4/2.
//
// A line of length L is owned by TPL = L/R threads; thread t holds the R
// elements at positions t + s*TPL (s = 0..R-1) in registers.  Each stage
// reads its butterflies' inputs from those registers, applies the stage
// twiddles, does a radix-r DFT in registers and scatters the outputs to LDS
// in Stockham order; after a barrier every thread re-reads positions
// t + s*TPL, which are exactly the inputs of its next-stage butterflies (r
// always divides R).  After the last stage the line sits in LDS in natural
// order and the registers again hold positions t + s*TPL.
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
  cx<T> w = tw[j];
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

// One Stockham stage with span NS, then recurse.  `lds` points at element 0
// of this thread's line; element p lives at lds[p * stride].  R elements
// per thread (a power of two, 2..8).
template <typename T, int L, int R, int S, int NS>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[R], cx<T>* lds,
                                           int stride, int t,
                                           const cx<T>* tw) {
  if constexpr (NS < L) {
    constexpr int TPL = L / R;
    constexpr int rem = L / NS;
    constexpr int r = (rem % R == 0) ? R : rem;
    constexpr int NB = R / r;
    constexpr int twshift = TW_LOG - ilog2c(NS * r);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int b = t + q * TPL;
      const int k = b & (NS - 1);
      cx<T> a[r];
#pragma unroll
      for (int s = 0; s < r; ++s) a[s] = v[q + s * NB];
      if constexpr (NS > 1) {
#pragma unroll
        for (int s = 1; s < r; ++s)
          a[s] = cmul(a[s], twid<S>(tw, (s * k) << twshift));
      }
      butterfly<r, S>(a);
      const int base = (b / NS) * NS * r + k;
#pragma unroll
      for (int s = 0; s < r; ++s) lds[(base + s * NS) * stride] = a[s];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = lds[(t + s * TPL) * stride];
    if constexpr (NS * r < L) __syncthreads();
    fft_stages<T, L, R, S, NS * r>(v, lds, stride, t, tw);
  }
}

// Full FFT of one line.  Precondition: v[s] holds element t + s*TPL and no
// thread still reads this line's LDS (callers place a barrier before).
// Postcondition: natural-order result in LDS and in v (positions t+s*TPL).
// Every thread of the block must call this (it contains barriers).
template <typename T, int L, int S, int R>
__device__ __forceinline__ void fft_line(cx<T> (&v)[R], cx<T>* lds,
                                         int stride, int t, const cx<T>* tw) {
  if constexpr (L == 1) {
    return;
  } else {
    fft_stages<T, L, R, S, 1>(v, lds, stride, t, tw);
  }
}

}  // namespace expdiag
