// Pass B: everything of one Exp-ParaDiag iteration that is pointwise in the
// spatial wavevector kappa, fused into one kernel per tile of C kappa
// columns x all Nt time rows.
//
// For each kappa (spectral state U^_l, l = 0..Nt-1 <-> slices 1..Nt):
//   residual   R_l = E U_{l-1} + c1 N_l + c2 N_{l-1} - U_l
//              (U_{-1} = u0^, N_{-1} = N_0; eq. pcond-1st-order with the
//               lagged nonlinearity of Sec. 6.2; ETD1: c1 = dt phi1, c2 = 0;
//               ETD2: c1 = dt(phi1+phi2), c2 = -dt phi2)
//   step (a)   Y_m = sum_l e^{+2 pi i ml/Nt} gamma_l R_l       (F Gamma_alpha)
//   step (b)   X_m = Y_m / (Nt (1 - lambda_m E))                 shifted solves
//   step (c)   S_l = gamma_l^{-1} sum_m e^{-2 pi i ml/Nt} X_m  (Gamma^-1 F^*)
//   update     U_l += S_l
// (Sec. 3, eq. exp_ParaDiag_steps; the unitary 1/sqrt(Nt) factors of F and
// F^* are folded into the single 1/Nt of step (b).)
//
// The time transforms are length-Nt Stockham FFTs held in registers and LDS
// (fft_core.hpp).  Norms use Parseval with the half-spectrum weight (1 for
// the k_last = 0 and Nyquist planes, 2 otherwise).  Each block writes its
// partial sums; ctl_reduce_kernel then reduces an instance's partials in a
// fixed order (so the result does not depend on scheduling) and advances
// its convergence state.  (Doing that in the last-arriving pass B block
// needs a device-scope release fence in every block, which on this GPU
// writes back L2 and costs more than the extra launch.)
#pragma once
#include "kernels_fft.hpp"

namespace expdiag {

typedef double dbl2 __attribute__((ext_vector_type(2)));

enum PassBMode : int {
  PB_ITERATE = 0,   // residual + precond + update of U
  PB_PRECOND = 1,   // Sout = Q_alpha^{-1} Rin
  PB_RESIDUAL = 2,  // Sout = R(U)
  PB_OPAPPLY = 3,   // Sout = Q_alpha^{-1} (Q - G'(U)) v, v in U, J in Nh
  PB_PRECRES = 4,   // Sout = Q_alpha^{-1} R(U), norms of R and of Sout
};

struct PassBArgs {
  cx<double>* U;          // [Nt][Nk]
  // [Nt][Nk] fp32 iterate of the bulk phase (mixed, d >= 2, first-order
  // radix pass B), or null: the bulk phase reads and writes it, the switch
  // iteration (the first fp64 one) reads it and writes U
  cx<float>* U32;
  const void* Nh;         // [Nt][Nk] fp64 N^ (or J for PB_OPAPPLY), or null
  const void* Nh32;       // [Nt][Nk] fp32 N^ of the mixed bulk phase
  const cx<double>* u0h;  // [Nk]
  const cx<double>* E;    // [Nk] e^{dt mu} (complex when L has advection)
  const cx<double>* c1;   // [Nk] nonlinear weights of the scheme
  const cx<double>* c2;   // [Nk]
  const double* gam;      // [Nt]
  const double* igam;     // [Nt]
  const cx<double>* lam;  // [Nt]
  const cx<double>* Rin;  // [Nt][Nk] (PB_PRECOND)
  cx<double>* Sout;       // [Nt][Nk] (every mode but PB_ITERATE)
  double* partials;       // [nblocks][4]
  Ctl* ctl;               // iterate mode: convergence state (else null)
  Ctl* hmirror;           // host-mapped copy of *ctl (nullable)
  double* hist;           // [max_iter][2] (rel, ||R||) history (nullable)
  const cx<double>* tw;
  const cx<double>* roots;  // e^{+2 pi i j/N}, j < N (EBDF dense transform)
  long Nk;
  int nh;
  int nonlinear;
  int etd2;
  int nblocks;
  double inv_ns;
  // IF1 (the nonlinear term of row l is N(u_l), not N(u_{l-1})): same_slice
  // keeps the row-0 term of the Jacobian product; the preconditioner is
  // Q_alpha - sigma I with sigma = `sigma` (single launches) or the control
  // block's value (iterations, jac_mode != 0).  jac_mode 1: after each
  // iteration sigma = jac_c[0] + jac_c[1] mean(u) + jac_c[2] mean(u^2) over
  // space-time (dt times the mean of N'(u)); the block holding kappa = 0
  // adds sum_l Re U^_l(0) as partial 3.  inv_ntns = 1 / (Nt Ns).
  int same_slice;
  int bdf_s;  // order s of an exponential BDF window (2..6), else 0
  int jac_mode;
  double sigma;
  double jac_c[3];
  double inv_ntns;
  // gamma_{s TPL} and 1/gamma_{s TPL}, s < R, of the radix-FFT pass B
  // (R = min(Nt, 4), TPL = Nt/R): row t + s TPL of a thread scales by
  // gamma_t gamma_{s TPL}
  double gstep[4];
  double igstep[4];
};

// C kappa columns per workgroup, TPL threads per column, four time rows per
// thread (radix-4 stages keep the registers within the occupancy below).
// Thread (c, t) = (tid % C, tid / C) and tile element (l, c) at LDS l*C + c,
// so every global access of a wavefront is a run of C adjacent kappa (256
// bytes).  (A layout with whole columns inside one wavefront needs only
// wavefront-level synchronisation, but splits each wavefront's global
// accesses into 64-byte runs and costs registers; it measured slower.)
template <int NT>
struct PassBShape {
  static constexpr int R = FftShape<NT, 4>::R;
  static constexpr int TPL = FftShape<NT, 4>::TPL;
  static constexpr int C = (256 / TPL) >= 4 ? 256 / TPL : 4;
  static constexpr int THREADS = C * TPL;
  static constexpr int LS = C;        // LDS row (complex slots)
  static constexpr int LDS = NT * C;  // complex elements of the tile
  // waves per SIMD the register budget targets: every load of a thread is
  // in flight at once, which needs 97-128 registers; at five waves the
  // spills cost more than the extra wave gains
  static constexpr int WAVES = 4;
};

// Sum NV doubles over the block; thread 0 writes them to out[0..NV).
// Sum four doubles over a wavefront.  The first two exchanges halve the
// values a lane carries (across 32 lanes a lane keeps values {0, 1} or
// {2, 3} and adds its partner's copies of them; across 16 it keeps one of
// the two), the last four sum that one value within each group of 16
// lanes: 7 exchanges of a double instead of 24.  Afterwards every lane of
// group g = lane / 16 holds the wavefront's total of value g.
__device__ __forceinline__ double wave_sum4(const double (&a)[4]) {
  const int lane = threadIdx.x & 63;
  const bool h32 = (lane & 32) != 0, h16 = (lane & 16) != 0;
  double k0 = h32 ? a[2] : a[0], k1 = h32 ? a[3] : a[1];
  const double s0 = h32 ? a[0] : a[2], s1 = h32 ? a[1] : a[3];
  k0 += __shfl_xor(s0, 32, 64);
  k1 += __shfl_xor(s1, 32, 64);
  double k = h16 ? k1 : k0;
  k += __shfl_xor(h16 ? k0 : k1, 16, 64);
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) k += __shfl_xor(k, off, 64);
  return k;
}

template <int NV, int THREADS>
__device__ __forceinline__ void block_sum(double (&acc)[NV], double* red,
                                          double* out) {
  constexpr int NW = (THREADS + 63) / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if constexpr (NV == 4) {
    static_assert(THREADS % 64 == 0, "whole wavefronts");
    const double k = wave_sum4(acc);
    __syncthreads();
    if ((lane & 15) == 0) red[wid * NV + (lane >> 4)] = k;
  } else {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double a = acc[j];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
      acc[j] = a;
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < NV; ++j) red[wid * NV + j] = acc[j];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double s = 0;
      for (int w = 0; w < NW; ++w) s += red[w * NV + j];
      out[j] = s;
    }
  }
}

// Convergence bookkeeping of one fixed-point iteration (thread 0 of the
// instance's reduction block).  tot = {||R||^2, ||S||^2, ||U||^2} (Parseval-weighted sums).
__device__ inline void advance_ctl(const PassBArgs& a, const double* tot) {
  Ctl* c = a.ctl;
  const double rn = sqrt(tot[0] * a.inv_ns);
  const double sn = sqrt(tot[1] * a.inv_ns);
  const double un = sqrt(tot[2] * a.inv_ns);
  const double rel = un > 0 ? sn / un : sn;
  const int it = c->iters + 1;
  c->iters = it;
  c->last_rel = rel;
  c->last_rnorm = rn;
  c->last_unorm = un;
  if (a.hist != nullptr && it <= c->max_iter) {
    a.hist[2 * (it - 1)] = rel;
    a.hist[2 * (it - 1) + 1] = rn;
  }
  const int phase0 = c->phase;
  int done = 0;
  if (a.jac_mode == 1) {
    const double mu1 = tot[3] * a.inv_ntns;
    const double mu2 = tot[2] * a.inv_ns * a.inv_ntns;
    c->sigma = a.jac_c[0] + a.jac_c[1] * mu1 + a.jac_c[2] * mu2;
  }
  if (!(rel == rel) || !(rn == rn) || rel > 1e300) {
    done = 2;
  } else if (c->phase == PH_BULK) {
    if (rel <= c->bulk_tol) {
      c->phase = PH_SWITCH;
      c->switch_iter = it;
    }
    if (it >= c->max_iter) done = 1;
  } else if (c->phase == PH_SWITCH) {
    // the first fp64 iteration (it has written the fp64 iterate)
    c->phase = PH_FP64;
    if (rel <= c->tol || it >= c->max_iter) done = 1;
  } else if (rel <= c->tol || it >= c->max_iter) {
    done = 1;
  }
  const bool publish = done != 0 || (it & 3) == 0 || c->phase != phase0;
  // read concurrently by the column blocks of the launch this may run in
  __hip_atomic_store(&c->done, done, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  if (a.hmirror != nullptr && publish) {
    volatile Ctl* m = a.hmirror;
    m->iters = it;
    m->phase = c->phase;
    m->switch_iter = c->switch_iter;
    m->last_rel = rel;
    m->last_rnorm = rn;
    m->last_unorm = un;
    m->done = done;
  }
}

// Every global load a thread needs is issued before the first value is
// used, and none sits behind a per-element branch (columns past Nk load
// column Nk-1 and are masked afterwards): global loads complete in issue
// order, so a load issued after the data loads, or a wait inside a loop,
// would cost another full memory latency.  The per-row tables are read
// once per thread: gamma_{t+s TPL} = gamma_t gamma_{s TPL} (the second
// factor is uniform, a scalar load) and lambda_{t+s TPL} = lambda_t
// e^{2 pi i s/R}.  Rows l-1 (of U, and of N^ for ETD2) come from the
// neighbouring threads through the LDS tile.
// Per-kappa symbol values: complex (L with advection) or their real parts
// (the tables' imaginary parts are zero), which keeps the registers of the
// real case.
template <bool CPLX>
struct SymOf {
  using T = cx<double>;
  static __device__ __forceinline__ T load(const cx<double>* p, long k) {
    return gld(p, k);
  }
  static __device__ __forceinline__ T zero() { return mk(0.0, 0.0); }
};
template <>
struct SymOf<false> {
  using T = double;
  static __device__ __forceinline__ T load(const cx<double>* p, long k) {
    return gld(reinterpret_cast<const double*>(p), 2 * k);
  }
  static __device__ __forceinline__ T zero() { return 0.0; }
};
__device__ __forceinline__ cx<double> smul(cx<double> a, double s) {
  return a * s;
}
__device__ __forceinline__ cx<double> smul(cx<double> a, cx<double> s) {
  return cmul(a, s);
}

// Uin / Uout: the iterate read and written in PB_ITERATE (fp32 or fp64;
// the arithmetic is fp64), the Krylov vector read in PB_OPAPPLY / the
// state in PB_RESIDUAL and PB_PRECRES (fp64); unused in PB_PRECOND.
template <int NT, int MODE, typename TN, bool CPLX, typename TUI = double,
          typename TUO = double>
__device__ __forceinline__ void passb_body(const PassBArgs& a, long lb,
                                           const TN* Nh, const cx<TUI>* Uin,
                                           cx<TUO>* Uout, cx<double>* lds,
                                           double* red) {
  using SY = SymOf<CPLX>;
  using SH = PassBShape<NT>;
  constexpr int R = SH::R;
  constexpr int TPL = SH::TPL;
  constexpr int C = SH::C;
  constexpr int LS = SH::LS;

  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const long Nk = a.Nk;
  const long kap = lb * C + c;
  const bool valid = kap < Nk;
  // Columns past Nk load column Nk - 1 (finite values of the same
  // arithmetic), carry them through unmasked, weigh 0 in the norms (pw) and
  // store nothing: every column's transform is independent of the others.
  const long kc = valid ? kap : Nk - 1;
  const int kl = static_cast<int>(kc) % a.nh;
  const double pw = (!valid) ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
  const cx<double> zero = mk(0.0, 0.0);

  // loads: data rows first, then the per-kappa and per-row tables.  An
  // fp32 iterate (the bulk phase) reads row l-1 of its own tile directly
  // (the block loads those lines anyway, so they come from the caches) in
  // place of the LDS exchange the fp64 variants make, which saves a trip
  // through LDS and a barrier where pass B is bound by its LDS traffic.
  constexpr bool GPREV = std::is_same<TUI, float>::value;
  cx<double> u[R];
  cx<TUI> uin[R];
  cx<TUI> upin[GPREV ? R : 1];
  cx<TN> nr[R];
  const cx<TN>* Nc = reinterpret_cast<const cx<TN>*>(Nh);
  const bool nl = MODE != PB_PRECOND && a.nonlinear;
  const bool two = nl && a.etd2;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int l = t + s * TPL;
    if constexpr (MODE == PB_PRECOND)
      u[s] = gld(a.Rin, l * Nk + kc);
    else
      uin[s] = gld(Uin, l * Nk + kc);
  }
  if constexpr (GPREV && MODE != PB_PRECOND) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int l = t + s * TPL;
      upin[s] = gld(Uin, (l > 0 ? l - 1 : 0) * Nk + kc);
    }
  }
  if (nl) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int l = t + s * TPL;
      nr[s] = gld(Nc, l * Nk + kc);
    }
  }
  const typename SY::T E = SY::load(a.E, kc);
  cx<double> first = zero;
  typename SY::T c1 = SY::zero(), c2 = SY::zero();
  if constexpr (MODE != PB_PRECOND && MODE != PB_OPAPPLY)
    first = gld(a.u0h, kc);
  if (nl) c1 = SY::load(a.c1, kc);
  if (two) c2 = SY::load(a.c2, kc);
  const double gam_t = gld(a.gam, t), igam_t = gld(a.igam, t);
  const cx<double> lam_t = gld(a.lam, t);
  double sigma = a.sigma;
  if (MODE == PB_ITERATE && a.jac_mode != 0) sigma = gld(&a.ctl->sigma, 0);
  constexpr int NST = fft_stage_count<NT, R>();
  cx<double> wst[NST > 1 ? NST : 2];
  fft_stage_twiddles<double, NT, R>(wst, t, a.tw);
  pin_loaded(wst);
  auto gam = [&](int s) { return s == 0 ? gam_t : gam_t * a.gstep[s]; };
  auto igam = [&](int s) { return s == 0 ? igam_t : igam_t * a.igstep[s]; };

  cx<double> v[R];
  double nrm_r = 0.0, nrm_s = 0.0, nrm_u = 0.0;

  if constexpr (MODE == PB_PRECOND) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      nrm_r += pw * norm2(u[s]);
      v[s] = u[s] * gam(s);
    }
  } else {
    // residual, U part (rows of U, or of the Krylov vector v for PB_OPAPPLY)
#pragma unroll
    for (int s = 0; s < R; ++s) {
      u[s] = cvt<double>(uin[s]);
      if constexpr (!GPREV) lds[(t + s * TPL) * LS + c] = u[s];
    }
    if constexpr (!GPREV) __syncthreads();
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int l = t + s * TPL;
      cx<double> prev;
      if constexpr (GPREV)
        prev = (l == 0) ? first : cvt<double>(upin[s]);
      else
        prev = (l == 0) ? first : lds[(l - 1) * LS + c];
      cx<double> n_cur = zero;
      if (nl && (MODE != PB_OPAPPLY || l >= 1 || a.same_slice))
        n_cur = cvt<double>(nr[s]);
      // PB_OPAPPLY, (Q - G'(U)) v: v_l - E v_{l-1} - (c1 J_l + c2 J_{l-1})
      // with J_l = FFT[N'(u_{l-1}) v_{l-1}] (J_0 = 0: u_0 is fixed); else
      // R_l = E U_{l-1} - U_l + c1 N_l + c2 N_{l-1}
      v[s] = (MODE == PB_OPAPPLY) ? u[s] - smul(prev, E) - smul(n_cur, c1)
                                  : smul(prev, E) - u[s] + smul(n_cur, c1);
      nr[s] = cvt<TN>(n_cur);  // masked row for the N_{l-1} exchange
    }
    if (two) {
      // ETD2: c2 N^_{l-1} with N^_{-1} := N^_0 (J_{-1} := 0 for PB_OPAPPLY)
      __syncthreads();
#pragma unroll
      for (int s = 0; s < R; ++s)
        lds[(t + s * TPL) * LS + c] = cvt<double>(nr[s]);
      __syncthreads();
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int l = t + s * TPL;
        const int lp = (l == 0) ? (MODE == PB_OPAPPLY ? -1 : 0) : l - 1;
        const cx<double> n_prev = lp < 0 ? zero : lds[lp * LS + c];
        v[s] = (MODE == PB_OPAPPLY) ? v[s] - smul(n_prev, c2)
                                    : v[s] + smul(n_prev, c2);
      }
    }
#pragma unroll
    for (int s = 0; s < R; ++s) {
      nrm_r += pw * norm2(v[s]);
      v[s] = v[s] * gam(s);
    }
    if constexpr (MODE == PB_RESIDUAL) {
      if (valid) {
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int l = t + s * TPL;
          gst(a.Sout, l * Nk + kap, v[s] * igam(s));
        }
      }
      double acc[4] = {nrm_r, 0.0, 0.0, 0.0};
      block_sum<4, SH::THREADS>(acc, red, a.partials + lb * 4);
      return;
    }
  }

  // step (a): forward time transform with the + sign.  Its exchanges
  // alternate between the tile's two LDS images starting with the second,
  // which the residual did not use, so no barrier precedes it; step (c)
  // continues the alternation, so none separates the two transforms.
  constexpr int XA = fft_exchanges<NT, R>();
  fft_line_pre<double, NT, 1, R, SH::LDS, 1>(v, lds + c, LS, t, wst);
  // step (b): shifted solves, 1/(Nt (1 - lambda_m E)), m = t + s TPL
#pragma unroll
  for (int s = 0; s < R; ++s) {
    cx<double> lam = lam_t;  // times e^{2 pi i s/R}
    if constexpr (R == 4) {
      if (s == 1) lam = mul_si<1>(lam_t);
      if (s == 2) lam = mk(-lam_t.x, -lam_t.y);
      if (s == 3) lam = mul_si<-1>(lam_t);
    } else if constexpr (R == 2) {
      if (s == 1) lam = mk(-lam_t.x, -lam_t.y);
    } else {
      static_assert(R == 1 || R == 2 || R == 4, "rotations for R <= 4");
    }
    const cx<double> z = smul(lam, E);
    const double dr = 1.0 - z.x - sigma, di = -z.y;
    // 1 / (NT |1 - lambda E - sigma|^2): the hardware reciprocal refined
    // by two Newton steps (within an ulp of the quotient; the denominator
    // is at least NT (1 - alpha^{1/Nt})^2 > 0, so no special cases)
    const double den = NT * (dr * dr + di * di);
    double inv = __builtin_amdgcn_rcp(den);
    inv = fma(fma(-den, inv, 1.0), inv, inv);
    inv = fma(fma(-den, inv, 1.0), inv, inv);
    v[s] = cmul(v[s], mk(dr * inv, -di * inv));
  }
  // step (c): inverse time transform with the - sign, then Gamma^{-1}.  A
  // fresh copy of the lane index makes it form its LDS addresses anew
  // rather than hold step (a)'s (the same ones) across step (b).
  int t2 = t;
  asm volatile("" : "+v"(t2));
  fft_line_pre<double, NT, -1, R, SH::LDS, (1 + XA) % 2>(v, lds + c, LS, t2,
                                                          wst);

  double sum0 = 0.0;  // sum_l Re U^_l(kappa = 0), for the IF1 mean Jacobian
  if constexpr (MODE == PB_ITERATE) {
    const bool k0 = a.jac_mode == 1 && kap == 0;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int l = t + s * TPL;
      const cx<double> sv = v[s] * igam(s);
      const cx<double> un = u[s] + sv;
      nrm_s += pw * norm2(sv);
      nrm_u += pw * norm2(un);
      if (k0) sum0 += un.x;
      if (valid) gst(Uout, l * Nk + kap, cvt<TUO>(un));
    }
  } else {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int l = t + s * TPL;
      const cx<double> sv = v[s] * igam(s);
      nrm_s += pw * norm2(sv);
      if (valid) gst(a.Sout, l * Nk + kap, sv);
    }
  }
  double acc[4] = {nrm_r, nrm_s, nrm_u, sum0};
  double tot[4];
  block_sum<4, SH::THREADS>(acc, red, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) a.partials[lb * 4 + j] = tot[j];
  }
}

template <int NT, int MODE, typename TN, bool CPLX>
__global__ void __launch_bounds__(PassBShape<NT>::THREADS,
                                  PassBShape<NT>::WAVES)
    passb_kernel(const PassBArgs* __restrict__ jobs,
                 const int* __restrict__ start, int njobs) {
  using SH = PassBShape<NT>;
  static_assert(SH::LDS * 2 >= ((SH::THREADS + 63) / 64) * 4,
                "reduction scratch fits the tile");
  __shared__ cx<double> lds[2 * SH::LDS];  // two images (fft_line_pre)
  double* red = reinterpret_cast<double*>(lds);
  // XCD-contiguous tiles: a tile's fp32 rows can be half a 128-byte line
  // (C = 8 columns at Nt = 128), whose other half the next tile reads
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int j = find_job(start, njobs, b);
  const PassBArgs a = jobs[j];  // by value: the kernel stores through a.U
  const long lb = b - start[j];
  if constexpr (MODE == PB_ITERATE) {
    const int ph = job_phase(a.ctl);
    if (ph < 0) return;
    if (lb == 0 && threadIdx.x == 0) {
      a.ctl->pending = 1;
      a.ctl->zstart = 0;  // the next pass A computes again
    }
    if (a.Nh32 != nullptr && ph == PH_BULK) {
      const float* n32 = static_cast<const float*>(a.Nh32);
      if (a.U32 != nullptr)
        passb_body<NT, MODE, float, CPLX, float, float>(a, lb, n32, a.U32,
                                                        a.U32, lds, red);
      else
        passb_body<NT, MODE, float, CPLX>(a, lb, n32, a.U, a.U, lds, red);
    } else if (a.U32 != nullptr && ph == PH_SWITCH) {
      passb_body<NT, MODE, double, CPLX, float, double>(
          a, lb, static_cast<const double*>(a.Nh), a.U32, a.U, lds, red);
    } else {
      passb_body<NT, MODE, double, CPLX>(
          a, lb, static_cast<const double*>(a.Nh), a.U, a.U, lds, red);
    }
  } else {
    passb_body<NT, MODE, TN, CPLX>(a, lb, static_cast<const TN*>(a.Nh), a.U,
                                   a.U, lds, red);
  }
}

// Convergence bookkeeping of one instance after a pass B: the fixed-order
// sum of its block partials, then advance_ctl.  Runs in one block of THREADS
// threads; does nothing unless a pass B has written partials since the
// last reduction (Ctl::pending), so it may be issued more often than
// needed.  Thread i adds partials i, i + THREADS, ... in that order (all of
// its loads issued before the first add), then the block sums the threads
// in a fixed tree.
template <int THREADS>
__device__ __forceinline__ void reduce_instance(const PassBArgs& a,
                                                double* red) {
  constexpr int UNROLL = 8;
  Ctl* ctl = a.ctl;
  if (gld(&ctl->done, 0) || !gld(&ctl->pending, 0)) return;
  const int nb = a.nblocks;
  const dbl2* pp = reinterpret_cast<const dbl2*>(a.partials);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b0 = threadIdx.x; b0 < nb; b0 += THREADS * UNROLL) {
    dbl2 lo[UNROLL], hi[UNROLL];
#pragma unroll
    for (int i = 0; i < UNROLL; ++i) {
      const int b = b0 + i * THREADS;
      lo[i] = b < nb ? gld(pp, 2 * b) : dbl2{0.0, 0.0};
      hi[i] = b < nb ? gld(pp, 2 * b + 1) : dbl2{0.0, 0.0};
    }
#pragma unroll
    for (int i = 0; i < UNROLL; ++i) {
      acc[0] += lo[i].x;
      acc[1] += lo[i].y;
      acc[2] += hi[i].x;
      acc[3] += hi[i].y;
    }
  }
  double tot[4];
  block_sum<4, THREADS>(acc, red, tot);
  if (threadIdx.x == 0) {
    ctl->pending = 0;
    advance_ctl(a, tot);
  }
}

// IF1 with a mean Jacobian: the first shift, sigma = jac_c[0] +
// jac_c[1] mean(u_0) + jac_c[2] mean(u_0^2), from the spectrum of u_0
// (mean(u_0) = Re u0^(0) / Ns, mean(u_0^2) = sum_k w_k |u0^_k|^2 / Ns^2).
// One block; fixed-order sums.
template <int THREADS>
__global__ void __launch_bounds__(THREADS)
    if1_sigma_init_kernel(const cx<double>* __restrict__ u0h, long Nk,
                          int nh, double inv_ns, double c0, double c1,
                          double c2, Ctl* ctl) {
  __shared__ double red[(THREADS / 64) * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long k = threadIdx.x; k < Nk; k += THREADS) {
    const int kl = static_cast<int>(k % nh);
    const double pw = (kl == 0 || kl == nh - 1) ? 1.0 : 2.0;
    acc[0] += pw * norm2(gld(u0h, k));
  }
  double tot[4];
  block_sum<4, THREADS>(acc, red, tot);
  if (threadIdx.x == 0) {
    const double mu1 = gld(u0h, 0).x * inv_ns;
    const double mu2 = tot[0] * inv_ns * inv_ns;
    ctl->sigma = c0 + c1 * mu1 + c2 * mu2;
  }
}

// Control-block initialisation on the stream (a kernel starts at once; a
// small host-to-device copy first waits for a copy engine).
__global__ void ctl_set_kernel(Ctl* __restrict__ dst, Ctl v) {
  if (threadIdx.x == 0) *dst = v;
}

// One block per job of a pass B job table.
constexpr int CTL_THREADS = 1024;

__global__ void __launch_bounds__(CTL_THREADS)
    ctl_reduce_kernel(const PassBArgs* __restrict__ jobs, int njobs) {
  __shared__ double red[(CTL_THREADS / 64) * 4];
  reduce_instance<CTL_THREADS>(jobs[blockIdx.x], red);
}

// The first inverse column stage of pass A (fp64, Uh -> T) with the
// previous iteration's convergence bookkeeping folded in: logical blocks
// [0, nred) each reduce one instance (red_jobs), the rest transform.  The
// transform does not depend on the convergence state (only pass B changes
// U), so it runs alongside the reduction; the later stages of the
// iteration, launched after this one, see the updated state.  A block may
// still transform an instance whose reduction in this launch finds it done:
// the result is never read.
template <int L, int S, int WD = 1>
__global__ void __launch_bounds__((ColShape<L, WD>::THREADS),
                                  (ColShape<L, WD>::WAVES))
    col_kernel_host(const ColJob* __restrict__ jobs,
                    const int* __restrict__ start, int njobs,
                    const PassBArgs* __restrict__ red_jobs, int nred,
                    const cx<double>* __restrict__ tw64) {
  __shared__ cx<double> lds[L * ColShape<L, WD>::LS];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  if (b < nred) {
    reduce_instance<(ColShape<L, WD>::THREADS)>(
        red_jobs[b], reinterpret_cast<double*>(lds));
    return;
  }
  const int cb = b - nred;
  const int i = find_job(start, njobs, cb);
  const ColJob jb = jobs[i];
  if (jb.ctl != nullptr &&
      (__hip_atomic_load(&jb.ctl->done, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT) ||
       __hip_atomic_load(&jb.ctl->zstart, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT)))
    return;
  col_body<double, L, S, double, double, WD>(jb, cb - start[i], tw64, lds);
}

template <int NT, int MODE, typename TN, bool CPLX>
__global__ void __launch_bounds__(PassBShape<NT>::THREADS,
                                  PassBShape<NT>::WAVES)
    passb_kernel1(PassBArgs a) {
  using SH = PassBShape<NT>;
  __shared__ cx<double> lds[2 * SH::LDS];  // two images (fft_line_pre)
  double* red = reinterpret_cast<double*>(lds);
  passb_body<NT, MODE, TN, CPLX>(a, xcd_block(blockIdx.x, gridDim.x),
                                 static_cast<const TN*>(a.Nh), a.U, a.U, lds,
                                 red);
}

// Fixed-order final reduction of per-block partials for the non-iterate
// modes: out[j] = inv_ns * sum_b partials[b][j].  One block of RED_THREADS
// threads; thread t adds blocks t, t + RED_THREADS, ... in that order, with
// RED_BATCH blocks' loads issued before the first add of each batch.
constexpr int RED_THREADS = 1024;
constexpr int RED_BATCH = 8;

__global__ void __launch_bounds__(RED_THREADS)
    reduce_kernel(const double* __restrict__ partials, int nblocks,
                  double inv_ns, double* __restrict__ out) {
  __shared__ double red[(RED_THREADS / 64) * 4];
  double acc[4] = {0, 0, 0, 0};
  for (int b0 = 0; b0 < nblocks; b0 += RED_THREADS * RED_BATCH) {
    double x[RED_BATCH][4];
#pragma unroll
    for (int q = 0; q < RED_BATCH; ++q) {
      const int b = b0 + threadIdx.x + q * RED_THREADS;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        x[q][j] = b < nblocks ? partials[static_cast<long>(b) * 4 + j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < RED_BATCH; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += x[q][j];
  }
  double tot[4];
  block_sum<4, RED_THREADS>(acc, red, tot);
  if (threadIdx.x != 0) return;
  for (int j = 0; j < 4; ++j) out[j] = tot[j] * inv_ns;
}

}  // namespace expdiag
