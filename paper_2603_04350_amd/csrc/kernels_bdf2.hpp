// Pass B of the second-order exponential BDF window (Sec. 4).
//
// The scheme u_n = 4/3 A u_{n-1} - 1/3 B u_{n-2}, B = A^2 (eq.
// 2nd_order_scheme) is started from u_1 = A u_0.  A tile row l = 0..Nt-1 is
// slice u_{l+1}.  Row 0 is the fixed start: its residual is E u0^ - U_0 and
// its preconditioner the identity.  Rows 1..Nt-1 are the unknowns
// v = (u_2..u_Nt) of eq. all_at_once_2ndorder; their residual is f_2 - R v
// with f_2 built from u0^ and E u0^, and R_alpha^{-1} (eq. pcond-2nd-order)
// is applied by steps (a)-(c) of eq. exp_ParaDiag_steps_2ndorder on
// N = Nt - 1 time points:
//   (a) Y_m = sum_j Wf[m][j] r_{j+1}, Wf[m][j] = gamma_j e^{+2 pi i mj/N}/N,
//       gamma_j = alpha^{j/N}
//   (b) X_m = Y_m / ((1 - lambda_m E)(1 - lambda_m E/3)),
//       lambda_m = alpha^{1/N} e^{2 pi i m/N}; the paper's shift
//       1 - 4/3 lambda_{0,m} E + 1/3 lambda_{1,m} E^2 with
//       lambda_{1,m} = lambda_{0,m}^2 factors this way
//   (c) s_{j+1} = sum_m Wi[j][m] X_m, Wi[j][m] = gamma_j^{-1} e^{-2 pi i mj/N}
// For Nt a power of two, N = Nt - 1 is not one, and the transform is the
// dense complex GEMM of kernels_dense.hpp: the host embeds the N x N matrices at
// row and column offset 1 of the Nt x Nt real-block operands (step (a)
// reads rows 1..N, step (c) writes them; row 0 and frequency N stay zero),
// which keeps the GEMM tiling of the Nt-point transform.
#pragma once
#include "kernels_dense.hpp"

namespace expdiag {

// MODE: PB_ITERATE (residual, precondition, update U), PB_RESIDUAL
// (Sout = residual), PB_PRECOND (Sout = P^{-1} Rin, in place allowed),
// PB_OPAPPLY (Sout = P^{-1} M v for v in U: row 0 of M v is v_0, rows
// j >= 1 are (R v)_j with the entries before v_2 taken as zero).
// P = diag(I, R_alpha).
template <int NT, int MODE>
__device__ __forceinline__ void passb_bdf2_body(const PassBArgs& a, long lb,
                                                double* lds, double* red) {
  constexpr int C = DENSE_C;
  constexpr int PER = NT * C / DENSE_THREADS > 0 ? NT * C / DENSE_THREADS : 1;
  double* Bm = lds;                  // [2NT][C]
  double* Ym = lds + 2 * NT * C;     // [2NT][C]
  cx<double>* Ut = reinterpret_cast<cx<double>*>(lds + 4 * NT * C);  // [NT][C]
  const long Nk = a.Nk;
  const long k0 = lb * C;
  const cx<double> zero = mk(0.0, 0.0);
  constexpr double c43 = 4.0 / 3.0, c13 = 1.0 / 3.0;
  double nrm_r = 0.0, nrm_s = 0.0, nrm_u = 0.0;

  // 1. rows of U (or v) into LDS: every row's residual needs the two before
  if constexpr (MODE != PB_PRECOND) {
    for (int e = threadIdx.x; e < NT * C; e += DENSE_THREADS) {
      const int l = e / C, c = e % C;
      const long kap = k0 + c;
      Ut[e] = kap < Nk ? gld(a.U, l * Nk + kap) : zero;
    }
    __syncthreads();
  }
  // 2. residual (or operator) rows; this thread keeps its own entries, the
  //    row-0 ones being their own preconditioned value
  cx<double> rk[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * DENSE_THREADS;
    rk[p] = zero;
    if (e >= NT * C) break;
    const int l = e / C, c = e % C;
    const long kap = k0 + c;
    const bool valid = kap < Nk;
    const int kl = static_cast<int>(kap % a.nh);
    const double pw = !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
    cx<double> r = zero;
    if (valid) {
      if constexpr (MODE == PB_PRECOND) {
        r = gld(a.Rin, l * Nk + kap);
      } else {
        const cx<double> E = gld(a.E, kap);
        const cx<double> E2 = cmul(E, E);
        const cx<double> u = Ut[e];
        // rows l-1 and l-2 (clamped; values, not addresses, are selected)
        const cx<double> q1 = Ut[(l >= 1 ? l - 1 : 0) * C + c];
        const cx<double> q2 = Ut[(l >= 2 ? l - 2 : 0) * C + c];
        if constexpr (MODE == PB_OPAPPLY) {
          r = u;
          if (l >= 2) r = r - cmul(q1, E * c43);
          if (l >= 3) r = r + cmul(q2, E2 * c13);
        } else {
          const cx<double> h0 = gld(a.u0h, kap);
          const cx<double> e1 = cmul(h0, E);  // u_1 = A u_0
          if (l == 0) {
            r = e1 - u;
          } else {
            const cx<double> p1 = l == 1 ? e1 : q1;
            const cx<double> p2 = l == 1 ? h0 : (l == 2 ? e1 : q2);
            r = cmul(p1, E * c43) - cmul(p2, E2 * c13) - u;
          }
        }
      }
    }
    rk[p] = r;
    nrm_r += pw * norm2(r);
    if constexpr (MODE == PB_RESIDUAL) {
      if (valid) a.Sout[l * Nk + kap] = r;
    } else {
      Bm[l * C + c] = r.x;
      Bm[(NT + l) * C + c] = r.y;
    }
  }
  if constexpr (MODE != PB_RESIDUAL) {
    __syncthreads();
    // 3. step (a) on MFMA
    dense_gemm<NT>(a.Wf, Bm, Ym);
    __syncthreads();
    // 4. step (b): both factors of the shifted second-order symbol
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * DENSE_THREADS;
      if (e >= NT * C) break;
      const int m = e / C, c = e % C;
      const long kap = k0 + c;
      const cx<double> E = kap < Nk ? gld(a.E, kap) : mk(0.0, 0.0);
      const cx<double> z = cmul(gld(a.lam, m), E);
      const cx<double> d = cmul(mk(1.0 - z.x, -z.y),
                                mk(1.0 - c13 * z.x, -c13 * z.y));
      const double inv = 1.0 / norm2(d);
      const cx<double> y = mk(Ym[m * C + c], Ym[(NT + m) * C + c]);
      const cx<double> x = cmulc(y, d) * inv;
      Bm[m * C + c] = x.x;
      Bm[(NT + m) * C + c] = x.y;
    }
    __syncthreads();
    // 5. step (c) on MFMA
    dense_gemm<NT>(a.Wi, Bm, Ym);
    __syncthreads();
    // 6. correction: row 0 keeps its residual
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * DENSE_THREADS;
      if (e >= NT * C) break;
      const int l = e / C, c = e % C;
      const long kap = k0 + c;
      const bool valid = kap < Nk;
      const int kl = static_cast<int>(kap % a.nh);
      const double pw =
          !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
      const cx<double> sv =
          l == 0 ? rk[p] : mk(Ym[l * C + c], Ym[(NT + l) * C + c]);
      nrm_s += pw * norm2(sv);
      if constexpr (MODE == PB_ITERATE) {
        // row 0 becomes E u0^ exactly rather than U_0 + (E u0^ - U_0)
        const cx<double> un =
            l == 0 ? (valid ? cmul(gld(a.u0h, kap), gld(a.E, kap)) : zero)
                   : Ut[e] + sv;
        nrm_u += pw * norm2(un);
        if (valid) a.U[l * Nk + kap] = un;
      } else {
        if (valid) a.Sout[l * Nk + kap] = sv;
      }
    }
  }
  double acc[4] = {nrm_r, nrm_s, nrm_u, 0.0};
  double tot[4];
  block_sum<4, DENSE_THREADS>(acc, red, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) a.partials[lb * 4 + j] = tot[j];
  }
}

// Job-table launch of the iteration (converged instances drop out).
template <int NT>
__global__ void __launch_bounds__(DENSE_THREADS)
    passb_bdf2_kernel(const PassBArgs* __restrict__ jobs,
                      const int* __restrict__ start, int njobs) {
  __shared__ double lds[dense_lds_doubles<NT>()];
  __shared__ double red[(DENSE_THREADS / 64) * 4];
  const int j = find_job(start, njobs);
  const PassBArgs a = jobs[j];
  const long lb = blockIdx.x - start[j];
  if (job_phase(a.ctl) < 0) return;
  if (lb == 0 && threadIdx.x == 0) a.ctl->pending = 1;
  passb_bdf2_body<NT, PB_ITERATE>(a, lb, lds, red);
}

template <int NT, int MODE>
__global__ void __launch_bounds__(DENSE_THREADS)
    passb_bdf2_kernel1(PassBArgs a) {
  __shared__ double lds[dense_lds_doubles<NT>()];
  __shared__ double red[(DENSE_THREADS / 64) * 4];
  passb_bdf2_body<NT, MODE>(a, blockIdx.x, lds, red);
}

// The same pass B when N = Nt - 1 is a power of two: the time transform is
// the radix FFT of kernels_passb.hpp (PassBShape<N>: C kappa columns per
// block, TPL threads per column, rows j = t + s TPL of the transform, which
// are window rows j + 1).  Rows j - 1 and j - 2 of the residual come from
// the neighbouring threads through the LDS tile; window row 0 is handled by
// the thread with t = 0 of each column.  All of a thread's global loads are
// issued before any is used (columns past Nk load column Nk - 1 and are
// masked afterwards).
template <int N, int MODE>
__device__ __forceinline__ void passb_bdf2_fft_body(const PassBArgs& a,
                                                    long lb, cx<double>* lds,
                                                    double* red) {
  using SH = PassBShape<N>;
  constexpr int R = SH::R;
  constexpr int TPL = SH::TPL;
  constexpr int C = SH::C;
  constexpr int LS = SH::LS;
  constexpr double c43 = 4.0 / 3.0, c13 = 1.0 / 3.0;
  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const long Nk = a.Nk;
  const long kap = lb * C + c;
  const bool valid = kap < Nk;
  const long kc = valid ? kap : Nk - 1;
  const int kl = static_cast<int>(kc) % a.nh;
  const double pw = !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
  const bool row0 = t == 0;  // this thread also owns window row 0
  const cx<double> zero = mk(0.0, 0.0);

  const cx<double>* in = MODE == PB_PRECOND ? a.Rin : a.U;
  cx<double> u[R];
#pragma unroll
  for (int s = 0; s < R; ++s) u[s] = gld(in, (t + s * TPL + 1) * Nk + kc);
  const cx<double> w0 = gld(in, kc);
  const cx<double> E = gld(a.E, kc);
  cx<double> h0 = zero;
  if constexpr (MODE == PB_ITERATE || MODE == PB_RESIDUAL) h0 = gld(a.u0h, kc);
  const double gam_t = gld(a.gam, t), igam_t = gld(a.igam, t);
  const cx<double> lam_t = gld(a.lam, t);
  constexpr int NST = fft_stage_count<N, R>();
  cx<double> wst[NST > 1 ? NST : 2];
  fft_stage_twiddles<double, N, R>(wst, t, a.tw);
  pin_loaded(wst);
  auto gam = [&](int s) { return s == 0 ? gam_t : gam_t * a.gstep[s]; };
  auto igam = [&](int s) { return s == 0 ? igam_t : igam_t * a.igstep[s]; };

  const cx<double> E2 = cmul(E, E);
  const cx<double> e1 = cmul(h0, E);  // u_1 = A u_0
  cx<double> v[R];
  cx<double> r0;  // window row 0: residual (or operator) row
  if constexpr (MODE == PB_PRECOND) {
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = u[s];
    r0 = w0;
  } else {
#pragma unroll
    for (int s = 0; s < R; ++s) lds[(t + s * TPL) * LS + c] = u[s];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int j = t + s * TPL;
      // rows j-1 and j-2 (clamped; values, not addresses, are selected)
      const cx<double> q1 = lds[(j >= 1 ? j - 1 : 0) * LS + c];
      const cx<double> q2 = lds[(j >= 2 ? j - 2 : 0) * LS + c];
      if constexpr (MODE == PB_OPAPPLY) {
        // (R v)_j with the entries before v_2 zero
        const cx<double> p1 = j >= 1 ? q1 : zero;
        const cx<double> p2 = j >= 2 ? q2 : zero;
        v[s] = u[s] - cmul(p1, E * c43) + cmul(p2, E2 * c13);
      } else {
        // f_2 - R v: row j needs u_{j+1} and u_j (u_1 = A u_0, u_0 given)
        const cx<double> p1 = j >= 1 ? q1 : e1;
        const cx<double> p2 = j >= 2 ? q2 : (j == 1 ? e1 : h0);
        v[s] = cmul(p1, E * c43) - cmul(p2, E2 * c13) - u[s];
      }
    }
    r0 = MODE == PB_OPAPPLY ? w0 : e1 - w0;
  }
  if (!valid) r0 = zero;
  double nrm_r = row0 ? pw * norm2(r0) : 0.0, nrm_s = 0.0, nrm_u = 0.0;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    if (!valid) v[s] = zero;
    nrm_r += pw * norm2(v[s]);
  }
  if constexpr (MODE == PB_RESIDUAL) {
    if (valid) {
#pragma unroll
      for (int s = 0; s < R; ++s)
        gst(a.Sout, (t + s * TPL + 1) * Nk + kap, v[s]);
      if (row0) gst(a.Sout, kap, r0);
    }
    double acc[4] = {nrm_r, 0.0, 0.0, 0.0};
    block_sum<4, SH::THREADS>(acc, red, a.partials + lb * 4);
    return;
  }
#pragma unroll
  for (int s = 0; s < R; ++s) v[s] = v[s] * gam(s);
  if constexpr (MODE != PB_PRECOND) __syncthreads();  // tile reads done

  // step (a): forward time transform with the + sign
  fft_line_pre<double, N, 1>(v, lds + c, LS, t, wst);
  // step (b): 1/(N (1 - lambda_m E)(1 - lambda_m E/3)), m = t + s TPL
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
    const cx<double> z = cmul(lam, E);
    const cx<double> d = cmul(mk(1.0 - z.x, -z.y),
                              mk(1.0 - c13 * z.x, -c13 * z.y));
    v[s] = cmulc(v[s], d) * (1.0 / (N * norm2(d)));
  }
  __syncthreads();
  // step (c): inverse time transform with the - sign, then Gamma^{-1}
  fft_line_pre<double, N, -1>(v, lds + c, LS, t, wst);

  if (row0) nrm_s += pw * norm2(r0);
  if constexpr (MODE == PB_ITERATE) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const cx<double> sv = v[s] * igam(s);
      const cx<double> un = u[s] + sv;
      nrm_s += pw * norm2(sv);
      nrm_u += pw * norm2(un);
      if (valid) gst(a.U, (t + s * TPL + 1) * Nk + kap, un);
    }
    // row 0 becomes E u0^ exactly rather than U_0 + (E u0^ - U_0)
    if (row0) {
      nrm_u += pw * norm2(valid ? e1 : zero);
      if (valid) gst(a.U, kap, e1);
    }
  } else {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const cx<double> sv = v[s] * igam(s);
      nrm_s += pw * norm2(sv);
      if (valid) gst(a.Sout, (t + s * TPL + 1) * Nk + kap, sv);
    }
    if (row0 && valid) gst(a.Sout, kap, r0);
  }
  double acc[4] = {nrm_r, nrm_s, nrm_u, 0.0};
  double tot[4];
  block_sum<4, SH::THREADS>(acc, red, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) a.partials[lb * 4 + j] = tot[j];
  }
}

template <int N>
__global__ void __launch_bounds__(PassBShape<N>::THREADS,
                                  PassBShape<N>::WAVES)
    passb_bdf2_fft_kernel(const PassBArgs* __restrict__ jobs,
                          const int* __restrict__ start, int njobs) {
  using SH = PassBShape<N>;
  __shared__ cx<double> lds[SH::LDS];
  double* red = reinterpret_cast<double*>(lds);
  const int j = find_job(start, njobs);
  const PassBArgs a = jobs[j];
  const long lb = blockIdx.x - start[j];
  if (job_phase(a.ctl) < 0) return;
  if (lb == 0 && threadIdx.x == 0) a.ctl->pending = 1;
  passb_bdf2_fft_body<N, PB_ITERATE>(a, lb, lds, red);
}

template <int N, int MODE>
__global__ void __launch_bounds__(PassBShape<N>::THREADS,
                                  PassBShape<N>::WAVES)
    passb_bdf2_fft_kernel1(PassBArgs a) {
  using SH = PassBShape<N>;
  __shared__ cx<double> lds[SH::LDS];
  double* red = reinterpret_cast<double*>(lds);
  passb_bdf2_fft_body<N, MODE>(a, blockIdx.x, lds, red);
}

// Slice u_1 = A u_0 of a spectral window (the fixed start of the scheme).
__global__ void bdf2_start_kernel(cx<double>* __restrict__ U,
                                  const cx<double>* __restrict__ u0h,
                                  const cx<double>* __restrict__ E, long Nk) {
  const long k = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < Nk) U[k] = cmul(u0h[k], E[k]);
}

}  // namespace expdiag
