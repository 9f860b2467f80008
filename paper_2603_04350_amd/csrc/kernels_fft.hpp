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
// Precision phases of an iteration (mixed precision): the bulk phase
// evaluates the residual with fp32 spatial FFTs and nonlinearity (and, for
// instances that keep their bulk iterate in fp32, stores the iterate in
// fp32); the switch iteration is the first fp64 one (it reads that fp32
// iterate and writes the fp64 one); the fp64 phase refines.  fp64
// instances run in PH_FP64 throughout.
enum : int { PH_BULK = 0, PH_SWITCH = 1, PH_FP64 = 2 };

struct Ctl {
  int done;      // 0 running, 1 finished (tolerance or max_iter), 2 diverged
  int phase;     // PH_BULK, PH_SWITCH or PH_FP64
  // 1 until the first pass B of a solve from the all-zero iterate: its
  // N^ rows of U's slices are zero (cleared at entry, as N(0) = 0), so that
  // iteration's pass-A stages have nothing to compute
  int zstart;
  int iters;     // iterations completed
  int max_iter;
  int pending;   // 1: pass B wrote block partials not yet reduced
  int switch_iter;  // mixed: the iteration after which the bulk phase
                    // ended (0 while it has not)
  double tol;       // ||S|| / ||U|| target
  double bulk_tol;  // switch from phase 0 to 1 below this
  double last_rel;
  double last_rnorm;
  double last_unorm;
  double sigma;     // IF1: Jacobian shift of the preconditioner (dt nbar)
};

// Phase of the job's instance (1 without a control block), or -1 when it
// has finished.
__device__ __forceinline__ int job_phase(const Ctl* c) {
  if (c == nullptr) return 1;
  typedef int i2 __attribute__((ext_vector_type(2)));
  const i2 dp = gld(reinterpret_cast<const i2*>(c), 0);  // {done, phase}
  return dp.x ? -1 : dp.y;
}

// job_phase for a pass-A stage of an iteration: also -1 while the
// instance's first iteration from the all-zero iterate has not reached its
// pass B (Ctl::zstart), whose N^ rows the entry has already zeroed
__device__ __forceinline__ int job_phase_a(const Ctl* c) {
  if (c == nullptr) return 1;
  typedef int i4 __attribute__((ext_vector_type(4)));
  const i4 d = gld(reinterpret_cast<const i4*>(c), 0);  // {done, phase, zstart}
  return (d.x || d.z) ? -1 : d.y;
}

// Values a thread has just issued loads for, marked as modified by an
// empty asm statement: the compiler then keeps them in registers instead of
// moving their loads next to the first use, where (loads completing in
// issue order) each would cost another memory latency.
template <typename T, int N>
__device__ __forceinline__ void pin_loaded(cx<T> (&w)[N]) {
#pragma unroll
  for (int i = 1; i < N; ++i) asm volatile("" : "+v"(w[i].x), "+v"(w[i].y));
}

// True when the job's instance still needs this work.  phase_req < 0: any
// phase.
__device__ __forceinline__ bool job_live(const Ctl* c, int phase_req) {
  if (c == nullptr) return true;
  if (gld(&c->done, 0)) return false;
  return phase_req < 0 || gld(&c->phase, 0) == phase_req;
}

// Job index of logical block b: largest j with start[j] <= b.  The result
// is the same for the whole block; readfirstlane makes that visible to the
// compiler so the job descriptor is fetched with scalar loads into scalar
// registers.
__device__ __forceinline__ int find_job(const int* __restrict__ start,
                                        int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}
__device__ __forceinline__ int find_job(const int* __restrict__ start,
                                        int njobs) {
  return find_job(start, njobs, blockIdx.x);
}

// Workgroups of a launch are dealt to the eight XCDs in turn (block b runs
// on XCD b % 8, each with its own L2).  This renumbering gives each XCD a
// contiguous range of logical blocks, so neighbouring tiles, which share
// the 128-byte lines at their edges, meet in the same L2.  A bijection of
// [0, G) for any G.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int q = G >> 3, rem = G & 7, x = b & 7;
  return x * q + (x < rem ? x : rem) + (b >> 3);
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
  // a row inside one wavefront synchronises only that wavefront
  static constexpr bool WAVE = TPR <= 64;
  // LDS slots per row: elements 0..M, padded one slot in nine
  static constexpr int LS = line_slots(M + 1, true);
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

// Forward half of a row: Z = FFT_M(z) of v (z_j = x_{2j} + i x_{2j+1}),
// then X_k = E_k + W^k O_k stored for k = 0..M (valid rows only).  The
// caller has synchronised so that nobody still reads this row's LDS.
// wst: stage twiddles (fft_stage_twiddles); wt = W^t, and W^{t + s*TPR} =
// wt e^{-i pi s/R} is formed where it is used (holding all R across the
// transform would cost 4R registers in fp64).
template <typename T, int M, typename TO, int R>
__device__ __forceinline__ void row_forward(const RowJob& jb, long row,
                                            bool valid, int t, cx<T> (&v)[R],
                                            cx<T>* lrow, const cx<T>* wst,
                                            cx<T> wt) {
  using S = RowShape<M>;
  constexpr int TPR = S::TPR;
  fft_stages<T, M, R, -1, 1, true, true, S::WAVE, 0, true>(
      v, mk<T>(1, 0), lrow, 1, t, wst);
  line_sync<S::WAVE>();
  if (!valid) return;
  cx<TO>* dst = static_cast<cx<TO>*>(jb.out) + row * (jb.out_pitch >> 1);
  cx<T> x0e, x0o;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int k = t + s * TPR;
    const cx<T> zk = v[s];
    const cx<T> zm = conj(lrow[slot<true>((M - k) & (M - 1))]);
    const cx<T> e = (zk + zm) * static_cast<T>(0.5);
    const cx<T> o = mul_si<-1>(zk - zm) * static_cast<T>(0.5);
    if (s == 0) {
      x0e = e;
      x0o = o;
    }
    const cx<T> wk = s == 0 ? wt : cmul(wt, eighth_root<T>(s * (8 / R)));
    const cx<T> x = e + cmul(wk, o);
    gst(dst, k, cvt<TO>(x));
  }
  if (t == 0) gst(dst, M, cvt<TO>(x0e - x0o));
}

// One block of the row transform: rows [lb*RPB, lb*RPB + RPB) of job `jb`.
// Row element k sits in LDS slot slot<true>(k) of its row; `lds` holds
// RPB * LS elements.  (Loading a second group of rows while the first is
// transformed, at the cost of the registers that holds, measured slower.)
template <typename T, int M, int MODE, typename TI, typename TO>
__device__ __forceinline__ void row_body(const RowJob& jb, long lb,
                                         const cx<T>* __restrict__ tw,
                                         cx<T>* lds) {
  using S = RowShape<M>;
  constexpr int R = S::R;
  constexpr int TPR = S::TPR;
  constexpr int wshift = TW_LOG - ilog2c(2 * M);
  const int rl = threadIdx.x / TPR;
  const int t = threadIdx.x % TPR;
  const long row = lb * S::RPB + rl;
  const bool valid = row < jb.nrows;
  // rows past the end read the last row (in bounds) and store nothing
  const long rowc = valid ? row : jb.nrows - 1;
  cx<T>* lrow = lds + rl * S::LS;
  const cx<TI>* src =
      static_cast<const cx<TI>*>(jb.in) + rowc * (jb.in_pitch >> 1);
  const T n1 = static_cast<T>(jb.n1), n2 = static_cast<T>(jb.n2),
          n3 = static_cast<T>(jb.n3);
  const T scale = static_cast<T>(jb.scale);
  cx<T> v[R];

  // every global load up front (loads complete in issue order, so a later
  // one would cost another memory latency): the row, then the twiddles.
  // W^k, k = t + s*TPR, is W^t e^{-i pi s/R}; the stage twiddles of both
  // transforms are the same (conjugated for the inverse).
  cx<TI> xin[R];
  cx<TI> xm_in = mk<TI>(0, 0);
#pragma unroll
  for (int s = 0; s < R; ++s) xin[s] = gld(src, t + s * TPR);
  if constexpr (MODE != ROW_R2C && MODE != ROW_NR2C) xm_in = gld(src, M);
  const cx<T> wt = gld(tw, t << wshift);
  constexpr int NST = fft_stage_count<M, R>();
  cx<T> wst[NST > 1 ? NST : 2];
  fft_stage_twiddles<T, M, R>(wst, t, tw);
  pin_loaded(wst);

  if constexpr (MODE == ROW_R2C || MODE == ROW_NR2C) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      cx<T> z = cvt<T>(xin[s]);
      if constexpr (MODE == ROW_NR2C) {
        z.x = nonlin(z.x, n1, n2, n3);
        z.y = nonlin(z.y, n1, n2, n3);
      }
      v[s] = z;
    }
  } else {
    // X_0..X_M of the half-spectrum row into LDS
#pragma unroll
    for (int s = 0; s < R; ++s)
      lrow[slot<true>(t + s * TPR)] = cvt<T>(xin[s]);
    // every lane of the row stores the same X_M: a store under t == 0
    // would let the compiler move the load behind the first wait
    lrow[slot<true>(M)] = cvt<T>(xm_in);
    line_sync<S::WAVE>();
    // Z_k = [(X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) W^{-k}] * scale
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int k = t + s * TPR;
      cx<T> xk = cvt<T>(xin[s]);  // this thread's own element
      cx<T> xm = lrow[slot<true>(M - k)];
      if (k == 0) {  // the k = 0 and Nyquist bins of a real row are real
        xk.y = 0;
        xm.y = 0;
      }
      const cx<T> wk = s == 0 ? wt : cmul(wt, eighth_root<T>(s * (8 / R)));
      const cx<T> e2 = xk + conj(xm);
      const cx<T> o2 = cmulc(xk - conj(xm), wk);
      v[s] = (e2 + mul_si<1>(o2)) * scale;
    }
    line_sync<S::WAVE>();
    fft_stages<T, M, R, 1, 1, true, false, S::WAVE, 0, true>(
        v, mk<T>(1, 0), lrow, 1, t, wst);
    // v[s] = z_j = x_{2j} + i x_{2j+1},  j = t + s*TPR
    if constexpr (MODE == ROW_C2R) {
      if (valid) {
        cx<TO>* dst = static_cast<cx<TO>*>(jb.out) + row * (jb.out_pitch >> 1);
#pragma unroll
        for (int s = 0; s < R; ++s) gst(dst, t + s * TPR, cvt<TO>(v[s]));
      }
      return;
    } else if constexpr (MODE == ROW_FUSED) {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        v[s].x = nonlin(v[s].x, n1, n2, n3);
        v[s].y = nonlin(v[s].y, n1, n2, n3);
      }
    } else {  // ROW_JVP
      const cx<TI>* ua =
          static_cast<const cx<TI>*>(jb.aux) + rowc * (jb.aux_pitch >> 1);
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const cx<T> u = cvt<T>(gld(ua, t + s * TPR));
        v[s].x *= dnonlin(u.x, n1, n2, n3);
        v[s].y *= dnonlin(u.y, n1, n2, n3);
      }
    }
    line_sync<S::WAVE>();
  }
  // a fresh copy of the lane index, so that the forward transform forms its
  // LDS addresses anew instead of keeping the inverse transform's (the same
  // addresses, which the compiler would otherwise hold across the
  // nonlinearity)
  int t2 = t;
  asm volatile("" : "+v"(t2));
  row_forward<T, M, TO>(jb, row, valid, t2, v, lrow, wst, wt);
}

// Complex rows of length M (the last axis of a complex state): row r of
// `out` (r * M complex elements in) = scale * FFT_S(row r of `in`); in
// place allowed (a block reads its rows before it writes).  Rows past
// nrows read the last row and store nothing.
template <int M, int S>
__global__ void __launch_bounds__(RowShape<M>::THREADS)
    row_c2c_kernel(const cx<double>* __restrict__ in, cx<double>* out,
                   long nrows, double scale,
                   const cx<double>* __restrict__ tw) {
  using SH = RowShape<M>;
  constexpr int R = SH::R;
  constexpr int TPR = SH::TPR;
  __shared__ cx<double> lds[SH::RPB * SH::LS];
  const int rl = threadIdx.x / TPR;
  const int t = threadIdx.x % TPR;
  const long row = static_cast<long>(blockIdx.x) * SH::RPB + rl;
  const bool valid = row < nrows;
  const cx<double>* src = in + (valid ? row : nrows - 1) * M;
  cx<double> v[R];
#pragma unroll
  for (int s = 0; s < R; ++s) v[s] = gld(src, t + s * TPR);
  constexpr int NST = fft_stage_count<M, R>();
  cx<double> wst[NST > 1 ? NST : 2];
  fft_stage_twiddles<double, M, R>(wst, t, tw);
  pin_loaded(wst);
  fft_stages<double, M, R, S, 1, true, false, SH::WAVE, 0, true>(
      v, mk(1.0, 0.0), lds + rl * SH::LS, 1, t, wst);
  if (!valid) return;
  cx<double>* dst = out + row * M;
#pragma unroll
  for (int s = 0; s < R; ++s) gst(dst, t + s * TPR, v[s] * scale);
}

// Job-table launch of one pass-A stage for instances in either precision
// phase: jobs[2i] is instance i's fp32 job (mixed-precision bulk phase),
// jobs[2i + 1] its fp64 job, and the instance's control block picks one, so
// an iteration costs one launch per stage in either phase.  Both bodies
// share one LDS tile (the fp32 one uses half of it).
template <int M, int MODE, typename TI0>
__global__ void __launch_bounds__(RowShape<M>::THREADS)
    row_kernel_mp(const RowJob* __restrict__ jobs,
                  const int* __restrict__ start, int njobs,
                  const cx<float>* __restrict__ tw32,
                  const cx<double>* __restrict__ tw64) {
  __shared__ cx<double> lds[RowShape<M>::RPB * RowShape<M>::LS];
  const int i = find_job(start, njobs);
  const long lb = blockIdx.x - start[i];
  const RowJob j1 = jobs[2 * i + 1];
  const int ph = job_phase_a(j1.ctl);
  if (ph < 0) return;
  if (ph == PH_BULK) {
    const RowJob jb = jobs[2 * i];
    row_body<float, M, MODE, TI0, float>(jb, lb, tw32,
                                         reinterpret_cast<cx<float>*>(lds));
  } else {
    row_body<double, M, MODE, double, double>(j1, lb, tw64, lds);
  }
}

// single job passed by value (per-call boundary transforms)
template <typename T, int M, int MODE, typename TI, typename TO>
__global__ void __launch_bounds__(RowShape<M>::THREADS)
    row_kernel1(RowJob jb, const cx<T>* __restrict__ tw) {
  __shared__ cx<T> lds[RowShape<M>::RPB * RowShape<M>::LS];
  if (!job_live(jb.ctl, jb.phase_req)) return;
  row_body<T, M, MODE, TI, TO>(jb, blockIdx.x, tw, lds);
}

// Job-table launch of a boundary-transform stage (entry and exit
// transforms of a batch): fp64, every job live, job j owning blocks
// [start[j], start[j+1]).
template <int M, int MODE>
__global__ void __launch_bounds__(RowShape<M>::THREADS)
    row_kernel_jt(const RowJob* __restrict__ jobs,
                  const int* __restrict__ start, int njobs,
                  const cx<double>* __restrict__ tw) {
  __shared__ cx<double> lds[RowShape<M>::RPB * RowShape<M>::LS];
  const int i = find_job(start, njobs);
  const RowJob jb = jobs[i];
  row_body<double, M, MODE, double, double>(jb, blockIdx.x - start[i], tw,
                                            lds);
}

// C adjacent columns per workgroup, at least 8 (a 128-byte run of fp64
// complex per row) while the tile of L*C complex fits 64 KiB of LDS, else
// 4; for L <= 256 the tile is 32 KiB in fp64, which lets five workgroups
// share a CU.  WAVES: the waves per SIMD that the LDS of one CU (160 KiB)
// allows, at most five (the register budget of the launch bounds).
// WD = 2: the wide variant of the same transform, 2C columns per workgroup
// (one of the autotuner's choices).
template <int L, int WD = 1>
struct ColShape {
  static constexpr int R = FftShape<L>::R;
  static constexpr int TPL = FftShape<L>::TPL;
  // columns per workgroup at least 8 while the tile is at most 64 KiB,
  // then 4 (up to L = 2048, 128 KiB) and 2 (L = 4096, 128 KiB)
  static constexpr int CMIN = L * 8 * 16 <= 65536 ? 8 : (L <= 2048 ? 4 : 2);
  static constexpr int C = WD * ((256 / TPL) >= CMIN ? 256 / TPL : CMIN);
  static constexpr int THREADS = C * TPL;
  static constexpr int LS = C;  // LDS row (complex slots)
  static constexpr int BLOCKS_LDS = 163840 / (L * C * 16);
  static constexpr int WAVES_LDS = BLOCKS_LDS * THREADS / 256;
  static constexpr int WAVES = WAVES_LDS < 1 ? 1 : (WAVES_LDS > 5 ? 5 : WAVES_LDS);
};

struct ColJob {
  const void* in;  // cx<TI>
  void* out;       // cx<TO>
  // fp64 job of the first pass-A stage of an instance whose bulk iterate
  // is fp32: that iterate (cx<float>), read instead of `in` in the switch
  // iteration; else null
  const void* in32;
  long outer, inner;
  double scale;
  const Ctl* ctl;
  int phase_req;
};

// Length-L transform along the middle axis of [outer][L][inner]; element
// (o, p, c) at (o*L + p)*inner + c.  out = scale * FFT_S(in); in-place safe.
// A job has outer * ceil(inner / C) blocks; lb < that count.
// `lds` holds L * LS elements.
template <typename T, int L, int S, typename TI, typename TO, int WD = 1>
__device__ __forceinline__ void col_body(const ColJob& jb, int lb,
                                         const cx<T>* __restrict__ tw,
                                         cx<T>* lds) {
  using SH = ColShape<L, WD>;
  constexpr int R = SH::R;
  constexpr int TPL = SH::TPL;
  constexpr int C = SH::C;
  const int inner = static_cast<int>(jb.inner);
  const int tiles = (inner + C - 1) / C;
  const int o = lb / tiles;
  const int tile = lb - o * tiles;
  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const int col = tile * C + c;
  const bool valid = col < inner;
  // columns past the edge read the last column (in bounds), store nothing
  const long base = static_cast<long>(o) * L * inner + (valid ? col : inner - 1);
  const cx<TI>* src = static_cast<const cx<TI>*>(jb.in) + base;
  cx<TI> xin[R];
#pragma unroll
  for (int s = 0; s < R; ++s) xin[s] = gld(src, (t + s * TPL) * inner);
  // stage twiddles issued with the data (loads complete in issue order)
  constexpr int NST = fft_stage_count<L, R>();
  cx<T> wst[NST > 1 ? NST : 2];
  fft_stage_twiddles<T, L, R>(wst, t, tw);
  pin_loaded(wst);
  cx<T> v[R];
#pragma unroll
  for (int s = 0; s < R; ++s) v[s] = cvt<T>(xin[s]);
  fft_stages<T, L, R, S, 1, false, false, false, 0, true>(
      v, mk<T>(1, 0), lds + c, SH::LS, t, wst);
  if (!valid) return;
  cx<TO>* dst = static_cast<cx<TO>*>(jb.out) + base;
  const T scale = static_cast<T>(jb.scale);
#pragma unroll
  for (int s = 0; s < R; ++s)
    gst(dst, (t + s * TPL) * inner, cvt<TO>(v[s] * scale));
}

// Job-table launch for instances in either precision phase (see
// row_kernel_mp): jobs[2i] fp32 (input type TI0, fp32 output), jobs[2i + 1]
// fp64.
template <int L, int S, typename TI0, int WD = 1>
__global__ void __launch_bounds__((ColShape<L, WD>::THREADS),
                                  (ColShape<L, WD>::WAVES))
    col_kernel_mp(const ColJob* __restrict__ jobs,
                  const int* __restrict__ start, int njobs,
                  const cx<float>* __restrict__ tw32,
                  const cx<double>* __restrict__ tw64) {
  __shared__ cx<double> lds[L * ColShape<L, WD>::LS];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = find_job(start, njobs, b);
  const int lb = b - start[i];
  const ColJob j1 = jobs[2 * i + 1];
  const int ph = job_phase_a(j1.ctl);
  if (ph < 0) return;
  if (ph == PH_BULK) {
    const ColJob jb = jobs[2 * i];
    col_body<float, L, S, TI0, float, WD>(jb, lb, tw32,
                                          reinterpret_cast<cx<float>*>(lds));
  } else if (ph == PH_SWITCH && j1.in32 != nullptr) {
    ColJob js = j1;
    js.in = j1.in32;
    col_body<double, L, S, float, double, WD>(js, lb, tw64, lds);
  } else {
    col_body<double, L, S, double, double, WD>(j1, lb, tw64, lds);
  }
}

// boundary-transform stage (see row_kernel_jt)
template <int L, int S>
__global__ void __launch_bounds__(ColShape<L>::THREADS, ColShape<L>::WAVES)
    col_kernel_jt(const ColJob* __restrict__ jobs,
                  const int* __restrict__ start, int njobs,
                  const cx<double>* __restrict__ tw) {
  __shared__ cx<double> lds[L * ColShape<L>::LS];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = find_job(start, njobs, b);
  const ColJob jb = jobs[i];
  col_body<double, L, S, double, double>(jb, b - start[i], tw, lds);
}

template <typename T, int L, int S, typename TI, typename TO>
__global__ void __launch_bounds__(ColShape<L>::THREADS, ColShape<L>::WAVES)
    col_kernel1(ColJob jb, const cx<T>* __restrict__ tw) {
  __shared__ cx<T> lds[L * ColShape<L>::LS];
  if (!job_live(jb.ctl, jb.phase_req)) return;
  col_body<T, L, S, TI, TO>(jb, xcd_block(blockIdx.x, gridDim.x), tw, lds);
}

}  // namespace expdiag
