// Pass B with the time transform as a dense complex GEMM on FP64 MFMA.
//
// Same computation as passb_body (kernels_passb.hpp), but steps (a) and (c)
// of eq. exp_ParaDiag_steps are applied to a tile of 16 kappa columns as
// dense products with the Nt x Nt complex matrices
//     Wf[m][l] = gamma_l e^{+2 pi i ml/Nt} / Nt,
//     Wi[l][m] = gamma_l^{-1} e^{-2 pi i ml/Nt},
// written as real block matrices [[Re, -Im], [Im, Re]] of size 2Nt x 2Nt
// (built on the host), so that [Y_re; Y_im] = Wf_big [R_re; R_im] is one
// real GEMM of (2Nt x 2Nt) by (2Nt x 16) on v_mfma_f64_16x16x4.  The
// pointwise shifted solve sits between the two GEMMs.
//
// MFMA f64 16x16x4 operand layout on gfx950 (64 lanes, checked on the
// device): A (16x4) lane i holds A[i%16][i/16]; B (4x16) lane i holds
// B[i/16][i%16]; result register j of lane i holds D[4j + i/16][i%16].
#pragma once
#include "kernels_passb.hpp"

namespace expdiag {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int DENSE_C = 16;        // kappa columns per workgroup
constexpr int DENSE_THREADS = 256;  // 4 waves

// D (2NT x 16, LDS, row-major, ld 16) = W (2NT x 2NT, global, row-major) *
// B (2NT x 16, LDS).  Waves split the 16-row output blocks.
template <int NT>
__device__ __forceinline__ void dense_gemm(const double* __restrict__ W,
                                           const double* Bm, double* Dm) {
  constexpr int K = 2 * NT;
  constexpr int RB = K / 16;  // 16-row output blocks
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  for (int ib = wave; ib < RB; ib += DENSE_THREADS / 64) {
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    const double* wrow = W + (ib * 16 + r) * K;
#pragma unroll 8
    for (int ks = 0; ks < K / 4; ++ks) {
      const double a = wrow[ks * 4 + q];
      const double b = Bm[(ks * 4 + q) * DENSE_C + r];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) Dm[(ib * 16 + 4 * j + q) * DENSE_C + r] = acc[j];
  }
}

// MODE: PB_ITERATE (residual, precondition, update) or PB_PRECOND.
template <int NT, int MODE, typename TN>
__device__ __forceinline__ void passb_dense_body(const PassBArgs& a, long lb,
                                                 const TN* Nh, double* lds,
                                                 double* red) {
  constexpr int C = DENSE_C;
  constexpr int PER = NT * C / DENSE_THREADS > 0 ? NT * C / DENSE_THREADS : 1;
  double* Bm = lds;                  // [2NT][C]
  double* Ym = lds + 2 * NT * C;     // [2NT][C]
  cx<double>* Ut = reinterpret_cast<cx<double>*>(lds + 4 * NT * C);  // [NT][C]
  const long Nk = a.Nk;
  const long k0 = lb * C;
  double nrm_r = 0.0, nrm_s = 0.0, nrm_u = 0.0;

  // 1. rows of U into LDS, then the residual as the real GEMM operand
  if constexpr (MODE == PB_ITERATE) {
    for (int e = threadIdx.x; e < NT * C; e += DENSE_THREADS) {
      const int l = e / C, c = e % C;
      const long kap = k0 + c;
      Ut[e] = kap < Nk ? a.U[l * Nk + kap] : mk(0.0, 0.0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * DENSE_THREADS;
    if (e >= NT * C) break;
    const int l = e / C, c = e % C;
    const long kap = k0 + c;
    const bool valid = kap < Nk;
    const int kl = static_cast<int>(kap % a.nh);
    const double pw = !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
    cx<double> r = mk(0.0, 0.0);
    if constexpr (MODE == PB_PRECOND) {
      if (valid) r = a.Rin[l * Nk + kap];
    } else {
      if (valid) {
        const cx<double> E = a.E[kap];
        const cx<double> prev = l == 0 ? a.u0h[kap] : Ut[(l - 1) * C + c];
        r = cmul(prev, E) - Ut[e];
        if (a.nonlinear) {
          const cx<TN>* Nc = reinterpret_cast<const cx<TN>*>(Nh);
          r = r + cmul(cvt<double>(Nc[l * Nk + kap]), a.c1[kap]);
          if (a.etd2)
            r = r + cmul(cvt<double>(Nc[(l == 0 ? 0 : l - 1) * Nk + kap]),
                         a.c2[kap]);
        }
      }
    }
    nrm_r += pw * norm2(r);
    Bm[l * C + c] = r.x;
    Bm[(NT + l) * C + c] = r.y;
  }
  __syncthreads();
  // 2. step (a): Y = Wf R on MFMA
  dense_gemm<NT>(a.Wf, Bm, Ym);
  __syncthreads();
  // 3. step (b): X_m = Y_m / (1 - lambda_m E), back into Bm
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * DENSE_THREADS;
    if (e >= NT * C) break;
    const int m = e / C, c = e % C;
    const long kap = k0 + c;
    const cx<double> E = kap < Nk ? a.E[kap] : mk(0.0, 0.0);
    const cx<double> z = cmul(a.lam[m], E);
    const double dr = 1.0 - z.x, di = -z.y;
    const double inv = 1.0 / (dr * dr + di * di);
    const cx<double> y = mk(Ym[m * C + c], Ym[(NT + m) * C + c]);
    const cx<double> x = cmul(y, mk(dr * inv, -di * inv));
    Bm[m * C + c] = x.x;
    Bm[(NT + m) * C + c] = x.y;
  }
  __syncthreads();
  // 4. step (c): S = Wi X on MFMA
  dense_gemm<NT>(a.Wi, Bm, Ym);
  __syncthreads();
  // 5. update / output
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * DENSE_THREADS;
    if (e >= NT * C) break;
    const int l = e / C, c = e % C;
    const long kap = k0 + c;
    const bool valid = kap < Nk;
    const int kl = static_cast<int>(kap % a.nh);
    const double pw = !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
    const cx<double> sv = mk(Ym[l * C + c], Ym[(NT + l) * C + c]);
    nrm_s += pw * norm2(sv);
    if constexpr (MODE == PB_ITERATE) {
      const cx<double> un = Ut[e] + sv;
      nrm_u += pw * norm2(un);
      if (valid) a.U[l * Nk + kap] = un;
    } else {
      if (valid) a.Sout[l * Nk + kap] = sv;
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

template <int NT>
constexpr int dense_lds_doubles() {
  return 6 * NT * DENSE_C;
}

template <int NT, int MODE, typename TN>
__global__ void __launch_bounds__(DENSE_THREADS)
    passb_dense_kernel(const PassBArgs* __restrict__ jobs,
                       const int* __restrict__ start, int njobs) {
  __shared__ double lds[dense_lds_doubles<NT>()];
  __shared__ double red[(DENSE_THREADS / 64) * 4];
  const int j = find_job(start, njobs);
  const PassBArgs a = jobs[j];
  const long lb = blockIdx.x - start[j];
  if constexpr (MODE == PB_ITERATE) {
    const int ph = job_phase(a.ctl);
    if (ph < 0) return;
    if (lb == 0 && threadIdx.x == 0) a.ctl->pending = 1;
    if (a.Nh32 != nullptr && ph == 0)
      passb_dense_body<NT, MODE, float>(
          a, lb, static_cast<const float*>(a.Nh32), lds, red);
    else
      passb_dense_body<NT, MODE, double>(
          a, lb, static_cast<const double*>(a.Nh), lds, red);
  } else {
    passb_dense_body<NT, MODE, TN>(a, lb, static_cast<const TN*>(a.Nh), lds,
                                   red);
  }
}

template <int NT, int MODE, typename TN>
__global__ void __launch_bounds__(DENSE_THREADS)
    passb_dense_kernel1(PassBArgs a) {
  __shared__ double lds[dense_lds_doubles<NT>()];
  __shared__ double red[(DENSE_THREADS / 64) * 4];
  passb_dense_body<NT, MODE, TN>(a, blockIdx.x, static_cast<const TN*>(a.Nh),
                                 lds, red);
}

}  // namespace expdiag
