// Krylov-vector kernels for GMRES on spectral space-time vectors.
//
// A Krylov vector is a half-spectrum space-time array [Nt][Nk] of complex
// fp64.  The real inner product of the physical fields it represents is,
// by Parseval, <x, y> = (1/Ns) sum_{l,kappa} w(kappa) Re(conj(x) y) with the
// half-spectrum weight w = 1 on the k_last = 0 and Nyquist planes, 2 else.
// All reductions are two-level with a fixed order, so results do not depend
// on scheduling.
#pragma once
#include "cx.hpp"

namespace expdiag {

constexpr int KRY_THREADS = 256;
constexpr int KRY_PER_THREAD = 4;
constexpr int KRY_PER_BLOCK = KRY_THREADS * KRY_PER_THREAD;

inline long krylov_blocks(long n) {
  long b = (n + KRY_PER_BLOCK - 1) / KRY_PER_BLOCK;
  return b < 1 ? 1 : b;
}

__device__ __forceinline__ double half_weight(long e, long Nk, int nh) {
  const long kap = e % Nk;
  const int kl = static_cast<int>(kap % nh);
  return (kl == 0 || kl == nh - 1) ? 1.0 : 2.0;
}

// Sum one double over the block; the result is valid in thread 0.
__device__ __forceinline__ double kry_block_sum(double a, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = a;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < KRY_THREADS / 64; ++w) s += red[w];
  }
  return s;
}

// part[i*ld + b] = block-partial <V_i, w> for i < nv; part[nv*ld + b] =
// block-partial <w, w>.  V_i = V + i*vstride (V unused when nv = 0).
// Vectors go in groups of KDOT_GROUP: the group's loads are all in flight
// before the first product, and one block reduction serves the group.
constexpr int KDOT_GROUP = 4;

__global__ void __launch_bounds__(KRY_THREADS)
    kdot_kernel(const cx<double>* __restrict__ V, long vstride, int nv,
                const cx<double>* __restrict__ w, long n, long Nk, int nh,
                double* __restrict__ part, int ld) {
  constexpr int NW = KRY_THREADS / 64;
  __shared__ double red[NW * KDOT_GROUP];
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  cx<double> wv[KRY_PER_THREAD];
  double pw[KRY_PER_THREAD];
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    const bool ok = e < n;
    wv[q] = ok ? w[e] : mk(0.0, 0.0);
    pw[q] = ok ? half_weight(e, Nk, nh) : 0.0;
  }
  for (int i0 = 0; i0 <= nv; i0 += KDOT_GROUP) {
    cx<double> x[KDOT_GROUP][KRY_PER_THREAD];
#pragma unroll
    for (int g = 0; g < KDOT_GROUP; ++g) {
      const int i = i0 + g;
#pragma unroll
      for (int q = 0; q < KRY_PER_THREAD; ++q) {
        const long e = base + threadIdx.x + q * KRY_THREADS;
        x[g][q] = mk(0.0, 0.0);
        if (i < nv && e < n) x[g][q] = V[i * vstride + e];
      }
    }
    double acc[KDOT_GROUP];
#pragma unroll
    for (int g = 0; g < KDOT_GROUP; ++g) {
      const int i = i0 + g;
      double a = 0.0;
      if (i < nv) {
#pragma unroll
        for (int q = 0; q < KRY_PER_THREAD; ++q) {
          const long e = base + threadIdx.x + q * KRY_THREADS;
          if (e < n)
            a += pw[q] * (x[g][q].x * wv[q].x + x[g][q].y * wv[q].y);
        }
      } else if (i == nv) {
#pragma unroll
        for (int q = 0; q < KRY_PER_THREAD; ++q) a += pw[q] * norm2(wv[q]);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
      acc[g] = a;
    }
    __syncthreads();  // the previous group's sums have been read
    if (lane == 0) {
#pragma unroll
      for (int g = 0; g < KDOT_GROUP; ++g) red[wid * KDOT_GROUP + g] = acc[g];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int g = 0; g < KDOT_GROUP; ++g) {
        const int i = i0 + g;
        if (i > nv) break;
        double sum = 0.0;
        for (int q = 0; q < NW; ++q) sum += red[q * KDOT_GROUP + g];
        part[static_cast<long>(i) * ld + blockIdx.x] = sum;
      }
    }
  }
}

// out[i] = scale * sum_b part[i*ld + b] (times vmul[i] when vmul is given),
// one block per i, fixed order:
// thread t adds partials t, t + KRED_THREADS, ... in that order, issuing
// KRED_BATCH of its loads before the first add of each batch (a dependent
// loop waited one memory latency per partial), then the block sums its
// threads in a fixed tree.
constexpr int KRED_THREADS = 1024;
constexpr int KRED_BATCH = 16;

__global__ void __launch_bounds__(KRED_THREADS)
    kreduce_kernel(const double* __restrict__ part, int nblocks, int ld,
                   double scale, const double* __restrict__ vmul,
                   double* __restrict__ out) {
  __shared__ double red[KRED_THREADS / 64];
  const int i = blockIdx.x;
  const double* row = part + static_cast<long>(i) * ld;
  double acc = 0.0;
  for (int b0 = 0; b0 < nblocks; b0 += KRED_THREADS * KRED_BATCH) {
    double x[KRED_BATCH];
#pragma unroll
    for (int q = 0; q < KRED_BATCH; ++q) {
      const int b = b0 + threadIdx.x + q * KRED_THREADS;
      x[q] = b < nblocks ? row[b] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < KRED_BATCH; ++q) acc += x[q];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < KRED_THREADS / 64; ++w) s += red[w];
    out[i] = vmul != nullptr ? s * scale * vmul[i] : s * scale;
  }
}

// w += sign * sum_{i<nv} coef[i] V_i ; optionally block partials of <w,w>
// (after the update) into part[b].
__global__ void __launch_bounds__(KRY_THREADS)
    kaxpy_kernel(cx<double>* __restrict__ w, const cx<double>* __restrict__ V,
                 long vstride, int nv, const double* __restrict__ coef,
                 double sign, long n, long Nk, int nh,
                 double* __restrict__ part, int ld) {
  __shared__ double red[KRY_THREADS / 64];
  __shared__ double cf[72];
  if (threadIdx.x < nv) cf[threadIdx.x] = sign * coef[threadIdx.x];
  __syncthreads();
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  // per element the terms are added in the order i = 0, 1, ...; two
  // vectors' loads are in flight at once
  cx<double> x[KRY_PER_THREAD];
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    x[q] = mk(0.0, 0.0);
    if (e < n) x[q] = w[e];
  }
  int i = 0;
  for (; i + 1 < nv; i += 2) {
    cx<double> y0[KRY_PER_THREAD], y1[KRY_PER_THREAD];
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      const long e = base + threadIdx.x + q * KRY_THREADS;
      y0[q] = mk(0.0, 0.0);
      y1[q] = mk(0.0, 0.0);
      if (e < n) {
        y0[q] = V[i * vstride + e];
        y1[q] = V[(i + 1) * vstride + e];
      }
    }
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      x[q] = x[q] + y0[q] * cf[i];
      x[q] = x[q] + y1[q] * cf[i + 1];
    }
  }
  if (i < nv) {
    cx<double> y0[KRY_PER_THREAD];
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      const long e = base + threadIdx.x + q * KRY_THREADS;
      y0[q] = mk(0.0, 0.0);
      if (e < n) y0[q] = V[i * vstride + e];
    }
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) x[q] = x[q] + y0[q] * cf[i];
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    if (e < n) {
      w[e] = x[q];
      if (part != nullptr) acc += half_weight(e, Nk, nh) * norm2(x[q]);
    }
  }
  if (part != nullptr) {
    const double s = kry_block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

// ---- Arnoldi with delayed reorthogonalisation (one reduction per step) --
// One pass over the basis V_0..V_{nv-1}, the pending vector u and (unless
// null) w = op(u): block partials of
//   rows i < nv: <V_i, u>;   rows nv + i: <V_i, w>;
//   row 2nv: <u, u>;  row 2nv + 1: <u, w>;  row 2nv + 2: <w, w>
// and, when w is null, rows i < nv: <V_i, u>, row nv: <u, u>.  The basis
// goes in groups of KDOT2_GROUP vectors (all their loads in flight before
// the first product, one block reduction per group); the group after the
// last basis vector carries the products of u and w.
constexpr int KDOT2_GROUP = 4;

__global__ void __launch_bounds__(KRY_THREADS)
    kdot2_kernel(const cx<double>* __restrict__ V, long vstride, int nv,
                 const cx<double>* __restrict__ u,
                 const cx<double>* __restrict__ w, long n, long Nk, int nh,
                 double* __restrict__ part, int ld) {
  constexpr int NW = KRY_THREADS / 64;
  constexpr int G = KDOT2_GROUP;
  constexpr int NV = 2 * G + 1;  // values reduced per group
  __shared__ double red[NW * NV];
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool hw = w != nullptr;
  cx<double> uv[KRY_PER_THREAD], wv[KRY_PER_THREAD];
  double pw[KRY_PER_THREAD];
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    const bool ok = e < n;
    uv[q] = ok ? u[e] : mk(0.0, 0.0);
    wv[q] = (ok && hw) ? w[e] : mk(0.0, 0.0);
    pw[q] = ok ? half_weight(e, Nk, nh) : 0.0;
  }
  // slot i < nv: basis vector i; slot nv: the products of u and w
  for (int i0 = 0; i0 <= nv; i0 += G) {
    cx<double> x[G][KRY_PER_THREAD];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int i = i0 + g;
#pragma unroll
      for (int q = 0; q < KRY_PER_THREAD; ++q) {
        const long e = base + threadIdx.x + q * KRY_THREADS;
        x[g][q] = mk(0.0, 0.0);
        if (i < nv && e < n) x[g][q] = V[i * vstride + e];
      }
    }
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int i = i0 + g;
      if (i < nv) {
#pragma unroll
        for (int q = 0; q < KRY_PER_THREAD; ++q) {
          acc[2 * g] += pw[q] * (x[g][q].x * uv[q].x + x[g][q].y * uv[q].y);
          acc[2 * g + 1] +=
              pw[q] * (x[g][q].x * wv[q].x + x[g][q].y * wv[q].y);
        }
      } else if (i == nv) {
#pragma unroll
        for (int q = 0; q < KRY_PER_THREAD; ++q) {
          acc[2 * g] += pw[q] * norm2(uv[q]);
          acc[2 * g + 1] += pw[q] * (uv[q].x * wv[q].x + uv[q].y * wv[q].y);
          acc[2 * G] += pw[q] * norm2(wv[q]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1)
        acc[k] += __shfl_down(acc[k], off, 64);
    }
    __syncthreads();  // the previous group's sums have been read
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) red[wid * NV + k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      auto sum = [&](int k) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += red[q * NV + k];
        return s;
      };
      const long b = blockIdx.x;
      for (int g = 0; g < G; ++g) {
        const int i = i0 + g;
        if (i < nv) {
          part[static_cast<long>(i) * ld + b] = sum(2 * g);
          if (hw) part[static_cast<long>(nv + i) * ld + b] = sum(2 * g + 1);
        } else if (i == nv) {
          if (hw) {
            part[static_cast<long>(2 * nv) * ld + b] = sum(2 * g);
            part[static_cast<long>(2 * nv + 1) * ld + b] = sum(2 * g + 1);
            part[static_cast<long>(2 * nv + 2) * ld + b] = sum(2 * G);
          } else {
            part[static_cast<long>(nv) * ld + b] = sum(2 * g);
          }
        }
      }
    }
  }
}

// The fused update of an Arnoldi step with delayed reorthogonalisation,
// u = V_j (pending), w = V_{j+1} (= op u):
//   q_j = (u - sum_{i<j} a_i V_i) / beta,
//   u'  = w / beta - sum_{i<j} z_i V_i - z_j q_j,
// q_j overwrites V_j and u' overwrites V_{j+1}.  cf = [a_0..a_{j-1},
// z_0..z_j, 1/beta] (device, 2j + 2 values, j <= 63).  Per element the
// terms are added in the order i = 0, 1, ...; two basis vectors' loads
// are in flight at once, each feeding both sums.
__global__ void __launch_bounds__(KRY_THREADS)
    kdcgs_update_kernel(cx<double>* __restrict__ V, long vstride, int j,
                        const double* __restrict__ coef, long n) {
  __shared__ double cf[2 * 64 + 2];
  if (threadIdx.x < 2 * j + 2) cf[threadIdx.x] = coef[threadIdx.x];
  __syncthreads();
  const double* ca = cf;
  const double* cz = cf + j;
  const double ib = cf[2 * j + 1];
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  cx<double> uq[KRY_PER_THREAD], wn[KRY_PER_THREAD];
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    uq[q] = mk(0.0, 0.0);
    wn[q] = mk(0.0, 0.0);
    if (e < n) {
      uq[q] = V[j * vstride + e];
      wn[q] = V[(j + 1) * vstride + e];
    }
  }
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) wn[q] = wn[q] * ib;
  int i = 0;
  for (; i + 1 < j; i += 2) {
    cx<double> y0[KRY_PER_THREAD], y1[KRY_PER_THREAD];
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      const long e = base + threadIdx.x + q * KRY_THREADS;
      y0[q] = mk(0.0, 0.0);
      y1[q] = mk(0.0, 0.0);
      if (e < n) {
        y0[q] = V[i * vstride + e];
        y1[q] = V[(i + 1) * vstride + e];
      }
    }
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      uq[q] = uq[q] - y0[q] * ca[i];
      uq[q] = uq[q] - y1[q] * ca[i + 1];
      wn[q] = wn[q] - y0[q] * cz[i];
      wn[q] = wn[q] - y1[q] * cz[i + 1];
    }
  }
  if (i < j) {
    cx<double> y0[KRY_PER_THREAD];
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      const long e = base + threadIdx.x + q * KRY_THREADS;
      y0[q] = mk(0.0, 0.0);
      if (e < n) y0[q] = V[i * vstride + e];
    }
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      uq[q] = uq[q] - y0[q] * ca[i];
      wn[q] = wn[q] - y0[q] * cz[i];
    }
  }
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    const cx<double> qj = uq[q] * ib;
    const cx<double> un = wn[q] - qj * cz[j];
    if (e < n) {
      V[j * vstride + e] = qj;
      V[(j + 1) * vstride + e] = un;
    }
  }
}

// ---- Complex Krylov vectors (complex states) ----------------------------
// A complex state's spectral vector is the full spectrum, and the inner
// product of the fields it represents is <x, y> = (1/Ns) sum conj(x) y
// (Parseval weight 1 on every entry): complex, where the real-state
// kernels above form its real part.
//
// kdot2c_kernel: block partials of, with G = KDOT2C_GROUP basis vectors per
// block reduction,
//   rows 2i, 2i+1: Re, Im <V_i, u>;  rows 2nv+2i, 2nv+2i+1: Re, Im <V_i, w>;
//   row 4nv: <u, u>;  rows 4nv+1, 4nv+2: Re, Im <u, w>;  row 4nv+3: <w, w>
// and, when w is null, rows 2i, 2i+1: <V_i, u>, row 2nv: <u, u>.
constexpr int KDOT2C_GROUP = 2;

__global__ void __launch_bounds__(KRY_THREADS)
    kdot2c_kernel(const cx<double>* __restrict__ V, long vstride, int nv,
                  const cx<double>* __restrict__ u,
                  const cx<double>* __restrict__ w, long n,
                  double* __restrict__ part, int ld) {
  constexpr int NW = KRY_THREADS / 64;
  constexpr int G = KDOT2C_GROUP;
  constexpr int NV = 4 * G + 4;  // values reduced per group
  __shared__ double red[NW * NV];
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool hw = w != nullptr;
  cx<double> uv[KRY_PER_THREAD], wv[KRY_PER_THREAD];
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    const bool ok = e < n;
    uv[q] = ok ? u[e] : mk(0.0, 0.0);
    wv[q] = (ok && hw) ? w[e] : mk(0.0, 0.0);
  }
  for (int i0 = 0; i0 <= nv; i0 += G) {
    cx<double> x[G][KRY_PER_THREAD];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int i = i0 + g;
#pragma unroll
      for (int q = 0; q < KRY_PER_THREAD; ++q) {
        const long e = base + threadIdx.x + q * KRY_THREADS;
        x[g][q] = mk(0.0, 0.0);
        if (i < nv && e < n) x[g][q] = V[i * vstride + e];
      }
    }
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int i = i0 + g;
      if (i < nv) {
#pragma unroll
        for (int q = 0; q < KRY_PER_THREAD; ++q) {
          const cx<double> a = x[g][q];
          acc[4 * g] += a.x * uv[q].x + a.y * uv[q].y;
          acc[4 * g + 1] += a.x * uv[q].y - a.y * uv[q].x;
          acc[4 * g + 2] += a.x * wv[q].x + a.y * wv[q].y;
          acc[4 * g + 3] += a.x * wv[q].y - a.y * wv[q].x;
        }
      } else if (i == nv) {
#pragma unroll
        for (int q = 0; q < KRY_PER_THREAD; ++q) {
          acc[4 * G] += norm2(uv[q]);
          acc[4 * G + 1] += uv[q].x * wv[q].x + uv[q].y * wv[q].y;
          acc[4 * G + 2] += uv[q].x * wv[q].y - uv[q].y * wv[q].x;
          acc[4 * G + 3] += norm2(wv[q]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1)
        acc[k] += __shfl_down(acc[k], off, 64);
    }
    __syncthreads();  // the previous group's sums have been read
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) red[wid * NV + k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      auto sum = [&](int k) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += red[q * NV + k];
        return s;
      };
      const long b = blockIdx.x;
      auto put = [&](long row, double v) { part[row * ld + b] = v; };
      for (int g = 0; g < G; ++g) {
        const int i = i0 + g;
        if (i < nv) {
          put(2 * i, sum(4 * g));
          put(2 * i + 1, sum(4 * g + 1));
          if (hw) {
            put(2 * nv + 2 * i, sum(4 * g + 2));
            put(2 * nv + 2 * i + 1, sum(4 * g + 3));
          }
        } else if (i == nv) {
          if (hw) {
            put(4 * nv, sum(4 * G));
            put(4 * nv + 1, sum(4 * G + 1));
            put(4 * nv + 2, sum(4 * G + 2));
            put(4 * nv + 3, sum(4 * G + 3));
          } else {
            put(2 * nv, sum(4 * G));
          }
        }
      }
    }
  }
}

// The fused update of a complex Arnoldi step (as kdcgs_update_kernel):
//   q_j = (u - sum_{i<j} a_i V_i) / beta,
//   u'  = w / beta - sum_{i<j} z_i V_i - z_j q_j,
// with complex a_i, z_i: cf = [a_0..a_{j-1}, z_0..z_j] as (re, im) pairs,
// then 1/beta (device, 4j + 3 values, j <= 63).
__global__ void __launch_bounds__(KRY_THREADS)
    kdcgs_updatec_kernel(cx<double>* __restrict__ V, long vstride, int j,
                         const double* __restrict__ coef, long n) {
  __shared__ double cf[4 * 64 + 4];
  for (int k = threadIdx.x; k < 4 * j + 3; k += KRY_THREADS)
    cf[k] = coef[k];
  __syncthreads();
  const cx<double>* ca = reinterpret_cast<const cx<double>*>(cf);
  const cx<double>* cz = ca + j;
  const double ib = cf[4 * j + 2];
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  cx<double> uq[KRY_PER_THREAD], wn[KRY_PER_THREAD];
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    uq[q] = mk(0.0, 0.0);
    wn[q] = mk(0.0, 0.0);
    if (e < n) {
      uq[q] = V[j * vstride + e];
      wn[q] = V[(j + 1) * vstride + e];
    }
  }
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) wn[q] = wn[q] * ib;
  for (int i = 0; i < j; ++i) {
    cx<double> y[KRY_PER_THREAD];
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      const long e = base + threadIdx.x + q * KRY_THREADS;
      y[q] = mk(0.0, 0.0);
      if (e < n) y[q] = V[i * vstride + e];
    }
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      uq[q] = uq[q] - cmul(y[q], ca[i]);
      wn[q] = wn[q] - cmul(y[q], cz[i]);
    }
  }
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    const cx<double> qj = uq[q] * ib;
    const cx<double> un = wn[q] - cmul(qj, cz[j]);
    if (e < n) {
      V[j * vstride + e] = qj;
      V[(j + 1) * vstride + e] = un;
    }
  }
}

// w += sum_{i<nv} coef_i V_i with complex coefficients (re, im pairs,
// nv <= 64); per element the terms are added in the order i = 0, 1, ...
__global__ void __launch_bounds__(KRY_THREADS)
    kaxpyc_kernel(cx<double>* __restrict__ w, const cx<double>* __restrict__ V,
                  long vstride, int nv, const double* __restrict__ coef,
                  long n) {
  __shared__ double cf[2 * 64];
  for (int k = threadIdx.x; k < 2 * nv; k += KRY_THREADS) cf[k] = coef[k];
  __syncthreads();
  const cx<double>* c = reinterpret_cast<const cx<double>*>(cf);
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  cx<double> x[KRY_PER_THREAD];
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    x[q] = e < n ? w[e] : mk(0.0, 0.0);
  }
  for (int i = 0; i < nv; ++i) {
#pragma unroll
    for (int q = 0; q < KRY_PER_THREAD; ++q) {
      const long e = base + threadIdx.x + q * KRY_THREADS;
      const cx<double> y = e < n ? V[i * vstride + e] : mk(0.0, 0.0);
      x[q] = x[q] + cmul(y, c[i]);
    }
  }
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    if (e < n) w[e] = x[q];
  }
}

// out = in * s (out may equal in)
__global__ void __launch_bounds__(KRY_THREADS)
    kscale_kernel(cx<double>* out, const cx<double>* in, double s, long n) {
  const long e = static_cast<long>(blockIdx.x) * KRY_THREADS + threadIdx.x;
  if (e < n) out[e] = in[e] * s;
}

// ---- BiCGStab (Table cpu_time_combined's preconditioned BiCGStab) -------
// Scalars live on the device in one array k[] so that an iteration needs a
// single host synchronisation (its convergence test): the reductions write
// the inner products, bicg_coef_kernel turns them into alpha, omega, beta,
// and the vector kernels read those.
enum {
  BI_RV = 0,      // <r^, v>   (kdot with V = r^, w = v; [1] is <v, v>)
  BI_SS = 2,      // <s, s>
  BI_ST = 3,      // <s, t>    (kdot with V = s, w = t; [4] is <t, t>)
  BI_TT = 4,
  BI_RHR = 5,     // <r^, r>   (after the x, r update; [6] is <r, r>)
  BI_RR = 6,
  BI_RHO = 8,     // rho = <r^, r> of the previous iteration
  BI_ALPHA = 9,
  BI_OMEGA = 10,
  BI_BETA = 11,
  BI_SLOTS = 12
};

// phase 0: alpha = rho / <r^, v>
// phase 1: omega = <s, t> / <t, t>, or 0 when ||s||^2 <= stop2 (the
//          iteration ends at x + alpha p, as BiCGStab's half-step exit)
// phase 2: beta = (<r^, r> / rho)(alpha / omega), rho = <r^, r>
__global__ void bicg_coef_kernel(double* __restrict__ k, int phase,
                                 double stop2) {
  if (threadIdx.x != 0) return;
  if (phase == 0) {
    k[BI_ALPHA] = k[BI_RHO] / k[BI_RV];
  } else if (phase == 1) {
    k[BI_OMEGA] = k[BI_SS] <= stop2 ? 0.0 : k[BI_ST] / k[BI_TT];
  } else {
    const double om = k[BI_OMEGA];
    k[BI_BETA] = om == 0.0 ? 0.0 : (k[BI_RHR] / k[BI_RHO]) * (k[BI_ALPHA] / om);
    k[BI_RHO] = k[BI_RHR];
  }
}

// s = r - alpha v; block partials of <s, s> into part[b]
__global__ void __launch_bounds__(KRY_THREADS)
    kbicg_s_kernel(cx<double>* __restrict__ s, const cx<double>* __restrict__ r,
                   const cx<double>* __restrict__ v,
                   const double* __restrict__ k, long n, long Nk, int nh,
                   double* __restrict__ part, int ld) {
  __shared__ double red[KRY_THREADS / 64];
  const double al = k[BI_ALPHA];
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  cx<double> rv[KRY_PER_THREAD], vv[KRY_PER_THREAD];
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    rv[q] = e < n ? r[e] : mk(0.0, 0.0);
    vv[q] = e < n ? v[e] : mk(0.0, 0.0);
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    if (e < n) {
      const cx<double> x = rv[q] - vv[q] * al;
      s[e] = x;
      acc += half_weight(e, Nk, nh) * norm2(x);
    }
  }
  const double t = kry_block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// x += alpha p + omega s; r = s - omega t; block partials of <r^, r> and
// <r, r> into part[b], part[ld + b]
__global__ void __launch_bounds__(KRY_THREADS)
    kbicg_xr_kernel(cx<double>* __restrict__ x, cx<double>* __restrict__ r,
                    const cx<double>* __restrict__ p,
                    const cx<double>* __restrict__ s,
                    const cx<double>* __restrict__ t,
                    const cx<double>* __restrict__ rh,
                    const double* __restrict__ k, long n, long Nk, int nh,
                    double* __restrict__ part, int ld) {
  __shared__ double red[KRY_THREADS / 64];
  const double al = k[BI_ALPHA], om = k[BI_OMEGA];
  const long base = static_cast<long>(blockIdx.x) * KRY_PER_BLOCK;
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int q = 0; q < KRY_PER_THREAD; ++q) {
    const long e = base + threadIdx.x + q * KRY_THREADS;
    if (e < n) {
      const cx<double> pe = p[e], se = s[e], te = t[e], he = rh[e];
      const cx<double> xe = x[e];
      x[e] = xe + pe * al + se * om;
      const cx<double> re = se - te * om;
      r[e] = re;
      const double w = half_weight(e, Nk, nh);
      a0 += w * (he.x * re.x + he.y * re.y);
      a1 += w * norm2(re);
    }
  }
  const double t0 = kry_block_sum(a0, red);
  const double t1 = kry_block_sum(a1, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = t0;
    part[ld + blockIdx.x] = t1;
  }
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(KRY_THREADS)
    kbicg_p_kernel(cx<double>* __restrict__ p, const cx<double>* __restrict__ r,
                   const cx<double>* __restrict__ v,
                   const double* __restrict__ k, long n) {
  const double be = k[BI_BETA], om = k[BI_OMEGA];
  const long e = static_cast<long>(blockIdx.x) * KRY_THREADS + threadIdx.x;
  if (e < n) p[e] = r[e] + (p[e] - v[e] * om) * be;
}

// zero fill (a plain kernel rather than a memset so that it can sit in a
// captured graph)
__global__ void __launch_bounds__(KRY_THREADS)
    kzero_kernel(cx<double>* out, long n) {
  const long e = static_cast<long>(blockIdx.x) * KRY_THREADS + threadIdx.x;
  if (e < n) out[e] = mk(0.0, 0.0);
}

}  // namespace expdiag
