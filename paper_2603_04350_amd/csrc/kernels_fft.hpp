// Batched spatial FFT kernels (periodic Fourier collocation).
//
// Spectral layout: a space-time slice of a real field on an n0 x .. x n_{d-1}
// grid is stored as its half spectrum, row-major [n0]..[n_{d-2}][nh] complex
// with nh = n_{d-1}/2 + 1 (the last index fastest), i.e. numpy's rfftn
// layout.  Forward transforms are unnormalised; inverse transforms carry the
// full 1/Ns factor in the row (last-axis) stage.
//
// Row kernel: one line of the last axis (n = 2M reals <-> M+1 complex) via a
// length-M complex FFT of z_j = x_{2j} + i x_{2j+1} and the standard
// even/odd split  X_k = E_k + W^k O_k,  W = e^{-2 pi i/n}.
// Column kernel: length-L transforms along a strided axis of an array viewed
// as [outer][L][inner]; a workgroup owns C adjacent `inner` columns so each
// global access is a contiguous run of C elements.
//
// Every launch walks a job table: job j owns blocks [start[j], start[j+1])
// of the grid, so one launch serves any number of instances of the same
// transform length (a single solve is a table of one job).  A job carries a
// pointer to its instance's control block and is skipped when that instance
// has finished or is not in the precision phase the job belongs to.
#pragma once
#include "fft_core.hpp"

namespace expdiag {

// Per-instance control block, device resident (kernels_passb.hpp updates it).
struct Ctl {
  int done;      // 0 running, 1 finished (tolerance or max_iter), 2 diverged
  int iters;     // iterations completed
  int max_iter;
  int phase;     // 0: fp32 bulk residual (mixed precision), 1: fp64
  double tol;       // ||S|| / ||U|| target
  double bulk_tol;  // switch from phase 0 to 1 below this
  double last_rel;
  double last_rnorm;
  double last_unorm;
};

// True when the job's instance still needs this work.  phase_req < 0: any
// phase.
__device__ __forceinline__ bool job_live(const Ctl* c, int phase_req) {
  if (c == nullptr) return true;
  if (c->done) return false;
  return phase_req < 0 || c->phase == phase_req;
}

// Job index of this block: largest j with start[j] <= blockIdx.x.  The
// result is the same for the whole block; readfirstlane makes that visible
// to the compiler so the job descriptor is fetched with scalar loads into
// scalar registers.
__device__ __forceinline__ int find_job(const int* __restrict__ start,
                                        int njobs) {
  int lo = 0, hi = njobs - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

enum RowMode : int {
  ROW_R2C = 0,    // real rows -> half spectrum
  ROW_C2R = 1,    // half spectrum -> real rows (scaled by `scale`)
  ROW_FUSED = 2,  // half spectrum -> real -> N(u) -> half spectrum
  ROW_NR2C = 3,   // real rows -> N(u) -> half spectrum
  ROW_JVP = 4,    // half spectrum v -> real -> N'(u) * v -> half spectrum
};

template <typename T>
__device__ __forceinline__ T nonlin(T u, T n1, T n2, T n3) {
  return u * (n1 + u * (n2 + u * n3));
}
template <typename T>
__device__ __forceinline__ T dnonlin(T u, T n1, T n2, T n3) {
  return n1 + u * (static_cast<T>(2) * n2 + u * static_cast<T>(3) * n3);
}

template <int M>
struct RowShape {
  static constexpr int R = FftShape<M>::R;
  static constexpr int TPR = FftShape<M>::TPL;
  static constexpr int RPB = TPR >= 256 ? 1 : 256 / TPR;
  static constexpr int THREADS = RPB * TPR;
  static constexpr int LS = M + 1;  // LDS complex slots per row
};

struct RowJob {
  const void* in;   // scalar array of the input type
  void* out;        // scalar array of the output type
  const void* aux;  // ROW_JVP: real field u (input type)
  long nrows, in_pitch, out_pitch, aux_pitch;  // pitches in scalars
  double scale;
  double n1, n2, n3;
  const Ctl* ctl;
  int phase_req;
};

// One block of the row transform: rows [lb*RPB, lb*RPB + RPB) of job `jb`.
template <typename T, int M, int MODE, typename TI, typename TO>
__device__ __forceinline__ void row_body(const RowJob& jb, long lb,
                                         const cx<T>* __restrict__ tw) {
  using S = RowShape<M>;
  constexpr int R = S::R;
  constexpr int TPR = S::TPR;
  constexpr int wshift = TW_LOG - ilog2c(2 * M);
  __shared__ cx<T> lds[S::RPB * S::LS];
  const int rl = threadIdx.x / TPR;
  const int t = threadIdx.x % TPR;
  const long row = lb * S::RPB + rl;
  const bool valid = row < jb.nrows;
  cx<T>* lrow = lds + rl * S::LS;
  const TI* in = static_cast<const TI*>(jb.in);
  TO* out = static_cast<TO*>(jb.out);
  const T n1 = static_cast<T>(jb.n1), n2 = static_cast<T>(jb.n2),
          n3 = static_cast<T>(jb.n3);
  const T scale = static_cast<T>(jb.scale);
  cx<T> v[R];

  if constexpr (MODE == ROW_R2C || MODE == ROW_NR2C) {
    const TI* src = in + row * jb.in_pitch;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int j = t + s * TPR;
      cx<T> z = mk<T>(0, 0);
      if (valid) z = cvt<T>(*reinterpret_cast<const cx<TI>*>(src + 2 * j));
      if constexpr (MODE == ROW_NR2C) {
        z.x = nonlin(z.x, n1, n2, n3);
        z.y = nonlin(z.y, n1, n2, n3);
      }
      v[s] = z;
    }
  } else {
    // load X_0..X_M of the half-spectrum row into LDS
    const TI* src = in + row * jb.in_pitch;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int k = t + s * TPR;
      cx<T> x = mk<T>(0, 0);
      if (valid) x = cvt<T>(*reinterpret_cast<const cx<TI>*>(src + 2 * k));
      lrow[k] = x;
    }
    if (t == 0) {
      cx<T> x = mk<T>(0, 0);
      if (valid) x = cvt<T>(*reinterpret_cast<const cx<TI>*>(src + 2 * M));
      lrow[M] = x;
    }
    __syncthreads();
    // Z_k = [(X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) W^{-k}] * scale
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int k = t + s * TPR;
      cx<T> xk = lrow[k];
      cx<T> xm = lrow[M - k];
      if (k == 0) {  // the k = 0 and Nyquist bins of a real row are real
        xk.y = 0;
        xm.y = 0;
      }
      const cx<T> e2 = xk + conj(xm);
      const cx<T> o2 = cmulc(xk - conj(xm), tw[k << wshift]);
      v[s] = (e2 + mul_si<1>(o2)) * scale;
    }
    __syncthreads();
    fft_line<T, M, 1>(v, lrow, 1, t, tw);
    // v[s] = z_j = x_{2j} + i x_{2j+1},  j = t + s*TPR
    if constexpr (MODE == ROW_C2R) {
      if (valid) {
        TO* dst = out + row * jb.out_pitch;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int j = t + s * TPR;
          *reinterpret_cast<cx<TO>*>(dst + 2 * j) = cvt<TO>(v[s]);
        }
      }
      return;
    } else if constexpr (MODE == ROW_FUSED) {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        v[s].x = nonlin(v[s].x, n1, n2, n3);
        v[s].y = nonlin(v[s].y, n1, n2, n3);
      }
    } else {  // ROW_JVP
      const TI* ua = static_cast<const TI*>(jb.aux) + row * jb.aux_pitch;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int j = t + s * TPR;
        cx<T> u = mk<T>(0, 0);
        if (valid) u = cvt<T>(*reinterpret_cast<const cx<TI>*>(ua + 2 * j));
        v[s].x *= dnonlin(u.x, n1, n2, n3);
        v[s].y *= dnonlin(u.y, n1, n2, n3);
      }
    }
    __syncthreads();
  }

  // forward: Z = FFT_M(z), then X_k = E_k + W^k O_k
  fft_line<T, M, -1>(v, lrow, 1, t, tw);
  if (!valid) return;
  TO* dst = out + row * jb.out_pitch;
  cx<T> x0e, x0o;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int k = t + s * TPR;
    const cx<T> zk = v[s];
    const cx<T> zm = conj(lrow[(M - k) & (M - 1)]);
    const cx<T> e = (zk + zm) * static_cast<T>(0.5);
    const cx<T> o = mul_si<-1>(zk - zm) * static_cast<T>(0.5);
    if (s == 0) {
      x0e = e;
      x0o = o;
    }
    const cx<T> x = e + cmul(tw[k << wshift], o);
    *reinterpret_cast<cx<TO>*>(dst + 2 * k) = cvt<TO>(x);
  }
  if (t == 0) *reinterpret_cast<cx<TO>*>(dst + 2 * M) = cvt<TO>(x0e - x0o);
}

template <typename T, int M, int MODE, typename TI, typename TO>
__global__ void __launch_bounds__(RowShape<M>::THREADS)
    row_kernel(const RowJob* __restrict__ jobs, const int* __restrict__ start,
               int njobs, const cx<T>* __restrict__ tw) {
  const int j = find_job(start, njobs);
  const RowJob jb = jobs[j];
  if (!job_live(jb.ctl, jb.phase_req)) return;
  row_body<T, M, MODE, TI, TO>(jb, blockIdx.x - start[j], tw);
}

// single job passed by value (per-call boundary transforms)
template <typename T, int M, int MODE, typename TI, typename TO>
__global__ void __launch_bounds__(RowShape<M>::THREADS)
    row_kernel1(RowJob jb, const cx<T>* __restrict__ tw) {
  if (!job_live(jb.ctl, jb.phase_req)) return;
  row_body<T, M, MODE, TI, TO>(jb, blockIdx.x, tw);
}

// C adjacent columns per workgroup; LDS of L*C complex (32 KiB in fp64 for
// L <= 512), which lets five workgroups share a CU.
template <int L>
struct ColShape {
  static constexpr int R = FftShape<L>::R;
  static constexpr int TPL = FftShape<L>::TPL;
  static constexpr int C = (256 / TPL) >= 4 ? 256 / TPL : 4;
  static constexpr int THREADS = C * TPL;
  static constexpr int LS = C;  // LDS row (complex slots)
};

struct ColJob {
  const void* in;  // cx<TI>
  void* out;       // cx<TO>
  long outer, inner;
  double scale;
  const Ctl* ctl;
  int phase_req;
};

// Length-L transform along the middle axis of [outer][L][inner]; element
// (o, p, c) at (o*L + p)*inner + c.  out = scale * FFT_S(in); in-place safe.
template <typename T, int L, int S, typename TI, typename TO>
__device__ __forceinline__ void col_body(const ColJob& jb, long lb,
                                         const cx<T>* __restrict__ tw) {
  using SH = ColShape<L>;
  constexpr int R = SH::R;
  constexpr int TPL = SH::TPL;
  constexpr int C = SH::C;
  __shared__ cx<T> lds[L * SH::LS];
  const long inner = jb.inner;
  const long tiles = (inner + C - 1) / C;
  const long o = lb / tiles;
  const long tile = lb % tiles;
  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const long col = tile * C + c;
  const bool valid = (col < inner) && (o < jb.outer);
  const cx<TI>* src = static_cast<const cx<TI>*>(jb.in) + o * L * inner + col;
  cx<T> v[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const long p = t + s * TPL;
    v[s] = valid ? cvt<T>(src[p * inner]) : mk<T>(0, 0);
  }
  fft_line<T, L, S>(v, lds + c, SH::LS, t, tw);
  if (!valid) return;
  cx<TO>* dst = static_cast<cx<TO>*>(jb.out) + o * L * inner + col;
  const T scale = static_cast<T>(jb.scale);
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const long p = t + s * TPL;
    dst[p * inner] = cvt<TO>(v[s] * scale);
  }
}

template <typename T, int L, int S, typename TI, typename TO>
__global__ void __launch_bounds__(ColShape<L>::THREADS, 5)
    col_kernel(const ColJob* __restrict__ jobs, const int* __restrict__ start,
               int njobs, const cx<T>* __restrict__ tw) {
  const int j = find_job(start, njobs);
  const ColJob jb = jobs[j];
  if (!job_live(jb.ctl, jb.phase_req)) return;
  col_body<T, L, S, TI, TO>(jb, blockIdx.x - start[j], tw);
}

template <typename T, int L, int S, typename TI, typename TO>
__global__ void __launch_bounds__(ColShape<L>::THREADS, 5)
    col_kernel1(ColJob jb, const cx<T>* __restrict__ tw) {
  if (!job_live(jb.ctl, jb.phase_req)) return;
  col_body<T, L, S, TI, TO>(jb, blockIdx.x, tw);
}

}  // namespace expdiag
