// Pass B of the order-s exponential BDF windows, s = 2..6 (Sec. 4 for s = 2,
// Sec. bdfs for s = 3..6).
//
// The scheme u_n = sum_{i=1..s} beta_i A^i u_{n-i} (eqs. 2nd_order_scheme,
// 3rd_order_scheme .. sixth_order_scheme) is started from u_m = A^m u_0,
// m < s.  A tile row l = 0..Nt-1 is slice u_{l+1}; rows l < o = s - 1 are
// the fixed starts (residual E^{l+1} u0^ - U_l, identity preconditioner).
// Rows o..Nt-1 are the unknowns v = (u_s..u_Nt) of the all-at-once system
// R_s v = f_s; their residual is f_s - R_s v with f_s built from u0^ and the
// start values.  Writing j = l - o, row l of it is
//     sum_{i=1..min(s,j)} beta_i E^i u_{l-i} + q_j E^{l+1} u0^ - u_l,
// where the start values enter only through q_j E^{l+1} u0^ (j < s):
// every such term is beta_i E^i E^{l+1-i} u0^, and sum_{i>j} beta_i = q_j
// below.  R_s^alpha has C_{i-1}^alpha = (C_0^alpha)^i, so steps (a)-(c) on
// N = Nt - o time points diagonalise it with eigenvalues lambda_m^i:
//   (a) Y_m = sum_j F[m][j] gamma_j r_{j+o}, F[m][j] = e^{+2 pi i mj/N}
//   (b) X_m = Y_m / (N d(lambda_m E)), d(z) = 1 - sum_i beta_i z^i
//       = (1 - z) sum_{k<s} q_k z^k, q_k = 1 - sum_{i<=k} beta_i
//       (d(1) = 0 because the beta_i sum to one; the factored form keeps the
//       1 - z of low modes free of the large coefficients' rounding)
//   (c) s_{j+o} = gamma_j^{-1} sum_m conj(F[m][j]) X_m
// For s = 2, d(z) = (1 - z)(1 - z/3).
//
// Two transforms: the DFT products on FP64 MFMA of kernels_dense.hpp for Nt
// a power of two (the N-point matrix placed at offset o of the Nt-row tile,
// its entries read from a table of the N roots of unity), and the radix FFT
// of kernels_passb.hpp when N is a power of two.
// SC is the order when it is fixed at compile time (the radix kernels of
// orders 2..4, where the run-time order cost 10-20%); SC = 0 reads it from
// PassBArgs::bdf_s and unrolls to six (radix orders 5 and 6, which spill
// when compiled in, and the dense kernels of orders 3..6).
#pragma once
#include "kernels_dense.hpp"

namespace expdiag {

// beta_i numerators over a common denominator (eqs. 2nd_order_scheme,
// 3rd_order_scheme, fourth_order_scheme, fifth_order_scheme,
// sixth_order_scheme)
constexpr int bdf_den(int s) {
  return s == 2 ? 3 : s == 3 ? 11 : s == 4 ? 25 : s == 5 ? 137 : 147;
}
constexpr int bdf_num(int s, int i) {
  constexpr int t2[2] = {4, -1};
  constexpr int t3[3] = {18, -9, 2};
  constexpr int t4[4] = {48, -36, 16, -3};
  constexpr int t5[5] = {300, -300, 200, -75, 12};
  constexpr int t6[6] = {360, -450, 400, -225, 72, -10};
  return s == 2   ? t2[i - 1]
         : s == 3 ? t3[i - 1]
         : s == 4 ? t4[i - 1]
         : s == 5 ? t5[i - 1]
                  : t6[i - 1];
}

struct BdfCoef {
  double beta[6];  // beta_1..beta_s (zero beyond s)
  double q[6];     // q_0..q_{s-1}: q_k = 1 - sum_{i<=k} beta_i
};

constexpr BdfCoef bdf_coef(int s) {
  BdfCoef c{};
  const int den = bdf_den(s);
  int acc = den;
  for (int i = 0; i < 6; ++i) {
    c.beta[i] = i < s ? static_cast<double>(bdf_num(s, i + 1)) / den : 0.0;
    c.q[i] = i < s ? static_cast<double>(acc) / den : 0.0;
    if (i < s) acc -= bdf_num(s, i + 1);
  }
  return c;
}

__constant__ BdfCoef kBdfCoef[5] = {bdf_coef(2), bdf_coef(3), bdf_coef(4),
                                    bdf_coef(5), bdf_coef(6)};

template <int SC>
__device__ __forceinline__ BdfCoef load_bdf_coef(int s) {
  if constexpr (SC > 0) {
    constexpr BdfCoef c = bdf_coef(SC);
    return c;
  } else {
    return kBdfCoef[s - 2];
  }
}

// q_k selected by value (k is per thread; no indexed private array)
template <int SMAX>
__device__ __forceinline__ double bdf_q_at(const BdfCoef& cf, int k) {
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < SMAX; ++i) r = k == i ? cf.q[i] : r;
  return r;
}

// E^p h for 1 <= p <= PMAX (p per thread)
template <int PMAX>
__device__ __forceinline__ cx<double> bdf_pow_times(cx<double> E, int p,
                                                    cx<double> h) {
  cx<double> r = h;
#pragma unroll
  for (int i = 1; i <= PMAX; ++i)
    if (i <= p) r = cmul(r, E);
  return r;
}

// sum_{i=1..min(s,j)} beta_i E^i p_i by Horner (p_i = row j - i)
template <int SMAX, typename Row>
__device__ __forceinline__ cx<double> bdf_history(const BdfCoef& cf, int s,
                                                  int j, cx<double> E,
                                                  Row row) {
  cx<double> acc = mk(0.0, 0.0);
#pragma unroll
  for (int i = SMAX; i >= 1; --i) {
    if (i > s) continue;
    const cx<double> p = row(i);  // clamped load, used only when i <= j
    acc = cmul(acc, E) + (i <= j ? p * cf.beta[i - 1] : mk(0.0, 0.0));
  }
  return cmul(acc, E);
}

// 1 / d(z), d(z) = (1 - z) sum_{k<s} q_k z^k, as conj(d) / |d|^2 * scale
template <int SMAX>
__device__ __forceinline__ cx<double> bdf_solve(const BdfCoef& cf, int s,
                                                cx<double> z, cx<double> y,
                                                double scale) {
  cx<double> qz = mk(0.0, 0.0);
#pragma unroll
  for (int k = SMAX - 1; k >= 0; --k) {
    if (k >= s) continue;
    qz = cmul(qz, z) + mk(cf.q[k], 0.0);
  }
  const cx<double> d = cmul(mk(1.0 - z.x, -z.y), qz);
  return cmulc(y, d) * (scale / norm2(d));
}

// LDS of the dense pass B: operand tile, iterate tile, the start rows'
// residuals, the roots, lambda, gamma and 1/gamma tables, E of the tile
template <int NT>
constexpr int bdf_dft_lds_doubles() {
  using SH = DftShape<NT>;
  return 2 * NT * SH::LD + 2 * NT * SH::C + 2 * 5 * SH::C + 2 * NT + 2 * NT +
         NT + NT + 2 * SH::C;
}

// MODE: PB_ITERATE (residual, precondition, update U), PB_RESIDUAL
// (Sout = residual), PB_PRECOND (Sout = P^{-1} Rin, in place allowed),
// PB_OPAPPLY (Sout = P^{-1} M v for v in U: rows l < o of M v are v_l, rows
// l >= o are (R_s v)_l with the entries before v_s taken as zero).
// P = diag(I, R_s^alpha).  A workgroup takes DftShape<NT>::C kappa
// columns; the residual phase gives each thread whole entries (row l,
// column c), the products and everything after them the accumulator layout
// of dft_units_n.
template <int NT, int SC, int MODE>
__device__ __forceinline__ void passb_bdf_body(const PassBArgs& a, long lb,
                                               double* lds, double* red) {
  using SH = DftShape<NT>;
  using EN = DftEntry<NT>;
  constexpr int C = SH::C;
  constexpr int LD = SH::LD;
  constexpr int SMAX = SC > 0 ? SC : 6;
  const int S = SC > 0 ? SC : a.bdf_s;
  const int o = S - 1;
  const int N = NT - o;
  const BdfCoef cf = load_bdf_coef<SC>(S);
  double* B = lds;                                              // [2NT][LD]
  cx<double>* Ut = reinterpret_cast<cx<double>*>(lds + 2 * NT * LD);  // [NT][C]
  cx<double>* rs = Ut + NT * C;                                 // [5][C]
  cx<double>* roots = rs + 5 * C;                               // [N]
  cx<double>* lamc = roots + NT;                                // [N]
  cx<double>* Ec = lamc + NT;                                   // [C]
  double* gml = reinterpret_cast<double*>(Ec + C);              // [N]
  double* igml = gml + NT;                                      // [N]
  const long Nk = a.Nk;
  const long k0 = lb * C;
  const cx<double> zero = mk(0.0, 0.0);
  double nrm_r = 0.0, nrm_s = 0.0, nrm_u = 0.0;

  if constexpr (MODE != PB_RESIDUAL) {
    for (int j = threadIdx.x; j < N; j += DENSE_THREADS) {
      roots[j] = gld(a.roots, j);
      lamc[j] = gld(a.lam, j);
      gml[j] = gld(a.gam, j);
      igml[j] = gld(a.igam, j);
    }
  }
  for (int c = threadIdx.x; c < C; c += DENSE_THREADS) {
    const long kap = k0 + c;
    Ec[c] = kap < Nk ? gld(a.E, kap) : zero;
  }
  // 1. rows of U (or v) into LDS: every row's residual needs the s before
  if constexpr (MODE != PB_PRECOND) {
#pragma unroll
    for (int p = 0; p < SH::PER; ++p) {
      const int e = threadIdx.x + p * DENSE_THREADS;
      const int l = e / C, c = e % C;
      const long kap = k0 + c;
      Ut[e] = kap < Nk ? gld(a.U, l * Nk + kap) : zero;
    }
  }
  __syncthreads();
  // 2. residual (or operator) rows; the unknown rows scaled by gamma as the
  //    operand of step (a), the start rows' (their own preconditioned
  //    value) kept aside and zero in the operand
#pragma unroll
  for (int p = 0; p < SH::PER; ++p) {
    const int e = threadIdx.x + p * DENSE_THREADS;
    const int l = e / C, c = e % C;
    const long kap = k0 + c;
    const bool valid = kap < Nk;
    const int kl = static_cast<int>((valid ? kap : 0) % a.nh);
    const double pw = !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
    cx<double> r = zero;
    if (valid) {
      if constexpr (MODE == PB_PRECOND) {
        r = gld(a.Rin, l * Nk + kap);
      } else {
        const cx<double> E = Ec[c];
        const cx<double> u = Ut[e];
        const int j = l - o;
        // rows l - i (clamped; values, not addresses, are selected)
        auto row = [&](int i) { return Ut[(l >= i ? l - i : 0) * C + c]; };
        if constexpr (MODE == PB_OPAPPLY) {
          r = j < 0 ? u : u - bdf_history<SMAX>(cf, S, j, E, row);
        } else {
          const cx<double> h0 = gld(a.u0h, kap);
          if (j < 0) {
            r = bdf_pow_times<SMAX - 1>(E, l + 1, h0) - u;
          } else {
            r = bdf_history<SMAX>(cf, S, j, E, row) - u;
            if (j < S)
              r = r + bdf_pow_times<2 * SMAX - 1>(E, l + 1, h0) *
                          bdf_q_at<SMAX>(cf, j);
          }
        }
      }
    }
    nrm_r += pw * norm2(r);
    if constexpr (MODE == PB_RESIDUAL) {
      if (valid) a.Sout[l * Nk + kap] = r;
    } else {
      if (l < o) rs[l * C + c] = r;
      const double g = l < o ? 0.0 : gml[l >= o ? l - o : 0];
      B[l * LD + c] = g * r.x;
      B[(NT + l) * LD + c] = g * r.y;
    }
  }
  if constexpr (MODE != PB_RESIDUAL) {
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, q = lane >> 4;
    const double inv_n = 1.0 / static_cast<double>(N);
    // 3. step (a) on MFMA (frequency m in row m), step (b) in registers;
    //    rows m >= N of the operand of step (c) are zero
    dbl4 acc[SH::PP][SH::CC][2];
    dft_units_n<NT, false>(B, roots, N, 0, N - o, acc);
    __syncthreads();  // every wave has read B: the X tile replaces it
#pragma unroll
    for (int i = 0; i < SH::PP; ++i) {
      const int p = wave % SH::WP + SH::WP * i;
#pragma unroll
      for (int jb = 0; jb < SH::CC; ++jb) {
        const int c = 16 * (wave / SH::WP + SH::G * jb) + r16;
#pragma unroll
        for (int e = 0; e < EN::N; ++e) {
          const int m = EN::row(p, e, q);
          cx<double> x = zero;
          if (m < N)
            x = bdf_solve<SMAX>(cf, S, cmul(lamc[m], Ec[c]),
                                EN::get(acc[i][jb], e), inv_n);
          B[m * LD + c] = x.x;
          B[(NT + m) * LD + c] = x.y;
        }
      }
    }
    __syncthreads();
    // 4. step (c) on MFMA (time row o + j in row o + j), then 1/gamma and
    //    the correction; start rows keep their residual
    dft_units_n<NT, true>(B, roots, N, N - o, 0, acc);
#pragma unroll
    for (int i = 0; i < SH::PP; ++i) {
      const int p = wave % SH::WP + SH::WP * i;
#pragma unroll
      for (int jb = 0; jb < SH::CC; ++jb) {
        const int c = 16 * (wave / SH::WP + SH::G * jb) + r16;
        const long kap = k0 + c;
        const bool valid = kap < Nk;
        const int kl = static_cast<int>((valid ? kap : 0) % a.nh);
        const double pw =
            !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
#pragma unroll
        for (int e = 0; e < EN::N; ++e) {
          const int l = EN::row(p, e, q);
          const cx<double> sv =
              l < o ? rs[(l < o ? l : 0) * C + c]
                    : EN::get(acc[i][jb], e) * igml[l >= o ? l - o : 0];
          nrm_s += pw * norm2(sv);
          if constexpr (MODE == PB_ITERATE) {
            // start rows become E^{l+1} u0^ exactly rather than U_l +
            // residual
            cx<double> un = Ut[l * C + c] + sv;
            if (l < o)
              un = valid ? bdf_pow_times<SMAX - 1>(Ec[c], l + 1,
                                                   gld(a.u0h, kap))
                         : zero;
            nrm_u += pw * norm2(un);
            if (valid) a.U[l * Nk + kap] = un;
          } else {
            if (valid) a.Sout[l * Nk + kap] = sv;
          }
        }
      }
    }
  }
  double accn[4] = {nrm_r, nrm_s, nrm_u, 0.0};
  double tot[4];
  block_sum<4, DENSE_THREADS>(accn, red, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) a.partials[lb * 4 + j] = tot[j];
  }
}

// Job-table launch of the iteration (converged instances drop out).
template <int NT, int SC>
__global__ void __launch_bounds__(DENSE_THREADS)
    passb_bdf_kernel(const PassBArgs* __restrict__ jobs,
                     const int* __restrict__ start, int njobs) {
  __shared__ double lds[bdf_dft_lds_doubles<NT>()];
  __shared__ double red[(DENSE_THREADS / 64) * 4];
  const int j = find_job(start, njobs);
  const PassBArgs a = jobs[j];
  const long lb = blockIdx.x - start[j];
  if (job_phase(a.ctl) < 0) return;
  if (lb == 0 && threadIdx.x == 0) a.ctl->pending = 1;
  passb_bdf_body<NT, SC, PB_ITERATE>(a, lb, lds, red);
}

template <int NT, int SC, int MODE>
__global__ void __launch_bounds__(DENSE_THREADS)
    passb_bdf_kernel1(PassBArgs a) {
  __shared__ double lds[bdf_dft_lds_doubles<NT>()];
  __shared__ double red[(DENSE_THREADS / 64) * 4];
  passb_bdf_body<NT, SC, MODE>(a, blockIdx.x, lds, red);
}

// The same pass B when N = Nt - o is a power of two: the time transform is
// the radix FFT of kernels_passb.hpp (PassBShape<N>: C kappa columns per
// block, TPL threads per column, rows j = t + r TPL of the transform, which
// are window rows j + o).  Rows j - 1 .. j - s of the residual come from the
// neighbouring threads through the LDS tile; the start rows are handled by
// the thread with t = 0 of each column.  All of a thread's global loads are
// issued before any is used (columns past Nk load column Nk - 1, carry its
// finite values through, weigh 0 in the norms and store nothing).
template <int N, int SC, int MODE>
__device__ __forceinline__ void passb_bdf_fft_body(const PassBArgs& a,
                                                   long lb, cx<double>* lds,
                                                   double* red) {
  using SH = PassBShape<N>;
  constexpr int R = SH::R;
  constexpr int TPL = SH::TPL;
  constexpr int C = SH::C;
  constexpr int LS = SH::LS;
  constexpr int SMAX = SC > 0 ? SC : 6;
  constexpr int OMAX = SMAX - 1;
  const int S = SC > 0 ? SC : a.bdf_s;
  const int o = S - 1;
  const BdfCoef cf = load_bdf_coef<SC>(S);
  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const long Nk = a.Nk;
  const long kap = lb * C + c;
  const bool valid = kap < Nk;
  const long kc = valid ? kap : Nk - 1;
  const int kl = static_cast<int>(kc) % a.nh;
  const double pw = !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
  const bool starts = t == 0;  // this thread also owns the start rows
  const cx<double> zero = mk(0.0, 0.0);

  const cx<double>* in = MODE == PB_PRECOND ? a.Rin : a.U;
  cx<double> u[R];
#pragma unroll
  for (int r = 0; r < R; ++r) u[r] = gld(in, (t + r * TPL + o) * Nk + kc);
  cx<double> w[OMAX];  // start rows (thread t = 0 only)
#pragma unroll
  for (int m = 0; m < OMAX; ++m)
    w[m] = starts && m < o ? gld(in, m * Nk + kc) : zero;
  const cx<double> E = gld(a.E, kc);
  cx<double> h0 = zero;
  if constexpr (MODE == PB_ITERATE || MODE == PB_RESIDUAL) h0 = gld(a.u0h, kc);
  const double gam_t = gld(a.gam, t), igam_t = gld(a.igam, t);
  const cx<double> lam_t = gld(a.lam, t);
  constexpr int NST = fft_stage_count<N, R>();
  cx<double> wst[NST > 1 ? NST : 2];
  fft_stage_twiddles<double, N, R>(wst, t, a.tw);
  pin_loaded(wst);
  auto gam = [&](int r) { return r == 0 ? gam_t : gam_t * a.gstep[r]; };
  auto igam = [&](int r) { return r == 0 ? igam_t : igam_t * a.igstep[r]; };

  cx<double> v[R];
  if constexpr (MODE == PB_PRECOND) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = u[r];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) lds[(t + r * TPL) * LS + c] = u[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = t + r * TPL;
      // rows j - i (clamped; values, not addresses, are selected)
      auto row = [&](int i) { return lds[(j >= i ? j - i : 0) * LS + c]; };
      const cx<double> hist = bdf_history<SMAX>(cf, S, j, E, row);
      if constexpr (MODE == PB_OPAPPLY) {
        v[r] = u[r] - hist;
      } else {
        v[r] = hist - u[r];
        if (j < S)
          v[r] = v[r] + bdf_pow_times<2 * SMAX - 1>(E, j + S, h0) *
                            bdf_q_at<SMAX>(cf, j);
      }
    }
  }
  double nrm_r = 0.0, nrm_s = 0.0, nrm_u = 0.0;
  // start rows, finished here (their preconditioner is the identity) so
  // that nothing of them stays live across the transform: residual (or
  // operator) row rs, and in PB_ITERATE the new value E^{m+1} u0^ exactly
  // rather than U_m + rs
  cx<double> em = h0;
#pragma unroll
  for (int m = 0; m < OMAX; ++m) {
    if (!starts || m >= o) continue;
    em = cmul(em, E);
    cx<double> rsm = w[m];
    if constexpr (MODE == PB_ITERATE || MODE == PB_RESIDUAL) rsm = em - w[m];
    nrm_r += pw * norm2(rsm);
    if constexpr (MODE != PB_RESIDUAL) nrm_s += pw * norm2(rsm);
    if constexpr (MODE == PB_ITERATE) {
      nrm_u += pw * norm2(em);
      if (valid) gst(a.U, m * Nk + kap, em);
    } else {
      if (valid) gst(a.Sout, m * Nk + kap, rsm);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) nrm_r += pw * norm2(v[r]);
  if constexpr (MODE == PB_RESIDUAL) {
    if (valid) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        gst(a.Sout, (t + r * TPL + o) * Nk + kap, v[r]);
    }
    double acc[4] = {nrm_r, 0.0, 0.0, 0.0};
    block_sum<4, SH::THREADS>(acc, red, a.partials + lb * 4);
    return;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = v[r] * gam(r);
  // step (a): forward time transform with the + sign; its exchanges
  // alternate between the two LDS images starting with the second, which
  // the residual's row reads did not use, and step (c) continues the
  // alternation (fft_line_pre), so neither needs a barrier before it
  constexpr int XA = fft_exchanges<N, R>();
  fft_line_pre<double, N, 1, R, SH::LDS, 1>(v, lds + c, LS, t, wst);
  // step (b): 1/(N d(lambda_m E)), m = t + r TPL
#pragma unroll
  for (int r = 0; r < R; ++r) {
    cx<double> lam = lam_t;  // times e^{2 pi i r/R}
    if constexpr (R == 4) {
      if (r == 1) lam = mul_si<1>(lam_t);
      if (r == 2) lam = mk(-lam_t.x, -lam_t.y);
      if (r == 3) lam = mul_si<-1>(lam_t);
    } else if constexpr (R == 2) {
      if (r == 1) lam = mk(-lam_t.x, -lam_t.y);
    } else {
      static_assert(R == 1 || R == 2 || R == 4, "rotations for R <= 4");
    }
    v[r] = bdf_solve<SMAX>(cf, S, cmul(lam, E), v[r], 1.0 / N);
  }
  // step (c): inverse time transform with the - sign, then Gamma^{-1}
  fft_line_pre<double, N, -1, R, SH::LDS, (1 + XA) % 2>(v, lds + c, LS, t,
                                                         wst);

  if constexpr (MODE == PB_ITERATE) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const cx<double> sv = v[r] * igam(r);
      const cx<double> un = u[r] + sv;
      nrm_s += pw * norm2(sv);
      nrm_u += pw * norm2(un);
      if (valid) gst(a.U, (t + r * TPL + o) * Nk + kap, un);
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const cx<double> sv = v[r] * igam(r);
      nrm_s += pw * norm2(sv);
      if (valid) gst(a.Sout, (t + r * TPL + o) * Nk + kap, sv);
    }
  }
  double acc[4] = {nrm_r, nrm_s, nrm_u, 0.0};
  double tot[4];
  block_sum<4, SH::THREADS>(acc, red, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) a.partials[lb * 4 + j] = tot[j];
  }
}

template <int N, int SC>
__global__ void __launch_bounds__(PassBShape<N>::THREADS,
                                  PassBShape<N>::WAVES)
    passb_bdf_fft_kernel(const PassBArgs* __restrict__ jobs,
                         const int* __restrict__ start, int njobs) {
  using SH = PassBShape<N>;
  __shared__ cx<double> lds[2 * SH::LDS];  // two images (fft_line_pre)
  double* red = reinterpret_cast<double*>(lds);
  const int j = find_job(start, njobs);
  const PassBArgs a = jobs[j];
  const long lb = blockIdx.x - start[j];
  if (job_phase(a.ctl) < 0) return;
  if (lb == 0 && threadIdx.x == 0) a.ctl->pending = 1;
  passb_bdf_fft_body<N, SC, PB_ITERATE>(a, lb, lds, red);
}

template <int N, int SC, int MODE>
__global__ void __launch_bounds__(PassBShape<N>::THREADS,
                                  PassBShape<N>::WAVES)
    passb_bdf_fft_kernel1(PassBArgs a) {
  using SH = PassBShape<N>;
  __shared__ cx<double> lds[2 * SH::LDS];  // two images (fft_line_pre)
  double* red = reinterpret_cast<double*>(lds);
  passb_bdf_fft_body<N, SC, MODE>(a, blockIdx.x, lds, red);
}

// Start slices u_m = A^m u_0, m = 1..o, of a spectral window (rows 0..o-1).
__global__ void bdf_start_kernel(cx<double>* __restrict__ U,
                                 const cx<double>* __restrict__ u0h,
                                 const cx<double>* __restrict__ E, long Nk,
                                 int o) {
  const long k = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= Nk) return;
  const cx<double> e = E[k];
  cx<double> v = u0h[k];
  for (int m = 0; m < o; ++m) {
    v = cmul(v, e);
    U[m * Nk + k] = v;
  }
}

}  // namespace expdiag
