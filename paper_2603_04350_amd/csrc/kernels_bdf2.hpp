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
// N is Nt - 1, never a power of two here, so the transform is the dense
// complex GEMM of kernels_dense.hpp: the host embeds the N x N matrices at
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
        const double E = gld(a.E, kap);
        const double E2 = E * E;
        const cx<double> u = Ut[e];
        if constexpr (MODE == PB_OPAPPLY) {
          r = u;
          if (l >= 2) r = r - Ut[(l - 1) * C + c] * (c43 * E);
          if (l >= 3) r = r + Ut[(l - 2) * C + c] * (c13 * E2);
        } else {
          const cx<double> h0 = gld(a.u0h, kap);
          const cx<double> e1 = h0 * E;  // u_1 = A u_0
          if (l == 0) {
            r = e1 - u;
          } else {
            const cx<double> p1 = l == 1 ? e1 : Ut[(l - 1) * C + c];
            const cx<double> p2 =
                l == 1 ? h0 : (l == 2 ? e1 : Ut[(l - 2) * C + c]);
            r = p1 * (c43 * E) - p2 * (c13 * E2) - u;
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
      const double E = kap < Nk ? gld(a.E, kap) : 0.0;
      const cx<double> z = gld(a.lam, m) * E;
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
            l == 0 ? (valid ? gld(a.u0h, kap) * gld(a.E, kap) : zero)
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

// Slice u_1 = A u_0 of a spectral window (the fixed start of the scheme).
__global__ void bdf2_start_kernel(cx<double>* __restrict__ U,
                                  const cx<double>* __restrict__ u0h,
                                  const double* __restrict__ E, long Nk) {
  const long k = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < Nk) U[k] = u0h[k] * E[k];
}

}  // namespace expdiag
