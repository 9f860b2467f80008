// Pass B with the time transform as dense products on FP64 MFMA.
//
// Same computation as passb_body (kernels_passb.hpp), with steps (a) and
// (c) of eq. exp_ParaDiag_steps applied as dense complex products on a
// tile of kappa columns, written as real GEMMs with block matrices
// [[Re, -Im], [Im, Re]] on v_mfma_f64_16x16x4.  The Gamma_alpha scaling is
// applied pointwise and the entries of the DFT matrix come from a table of
// roots of unity in LDS, so no matrix is stored or read: for first-order
// schemes the NT-point transform (passb_dft_body below), for the
// exponential BDFs (kernels_bdf.hpp) the N-point transform of the unknown
// rows, N = NT - s + 1.  The pointwise shifted solve sits between the two
// products.
//
// MFMA f64 16x16x4 operand layout on gfx950 (64 lanes, checked on the
// device): A (16x4) lane i holds A[i%16][i/16]; B (4x16) lane i holds
// B[i/16][i%16]; result register j of lane i holds D[4j + i/16][i%16].
#pragma once
#include "kernels_passb.hpp"

namespace expdiag {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int DENSE_THREADS = 256;  // 4 waves

// ---------------------------------------------------------------------
// First-order schemes: the time transform as DFT products on FP64 MFMA.
//
// Steps (a)-(c) of eq. exp_ParaDiag_steps on a tile of DftShape::C kappa
// columns: (a) row l of the residual is scaled by gamma_l and Y = F B with
// the NT x NT DFT matrix F[m][l] = w^{ml}, w = e^{+2 pi i/NT}; (b)
// X_m = Y_m / (NT (1 - lambda_m E)); (c) S_l = gamma_l^{-1} (conj(F) X)_l.
// Each complex product is one real GEMM with the block matrix
// [[Re F, -Im F], [Im F, Re F]] (conj(F): the signs of Im F flipped) on the
// stacked real and imaginary parts [2NT][C] of the tile in LDS.  The
// entries of F come from a table of the NT roots of unity (index ml mod NT)
// in LDS, so no NT x NT matrix is stored or read.
//
// A unit of a wave is a 16-column block of the tile with a "pair": the
// 16-row blocks of real and imaginary parts of the same 16 time
// frequencies (for NT = 8 one row block holds both: rows 0..7 real, 8..15
// imaginary).  Its lane then holds the real and imaginary part of the same
// complex entries in its accumulators, so step (b) and the update work in
// registers.
template <int NT>
struct DftShape {
  // kappa columns per workgroup: 64 KiB of LDS tiles for NT >= 32
  static constexpr int C = NT <= 32 ? 64 : 2048 / NT;
  static constexpr int LD = C + 2;      // LDS row of the real tile (doubles)
  static constexpr int NP = NT >= 16 ? NT / 16 : 1;  // row-block pairs
  static constexpr int CB = C / 16;     // column blocks
  static constexpr int WAVES = DENSE_THREADS / 64;
  // wave w takes the pairs p = w mod WP (PP of them) and the column blocks
  // cb = w / WP mod G (CC of them): per k-step it reads PP roots of unity
  // and CC operand values and issues 2 PP CC (NT = 8: PP CC) MFMAs
  static constexpr int WP = NP < WAVES ? NP : WAVES;
  static constexpr int G = WAVES / WP;
  static constexpr int PP = NP / WP;
  static constexpr int CC = CB / G;
  static constexpr int TILES = NT >= 16 ? 2 : 1;  // row blocks per pair
  static constexpr int PER = NT * C / DENSE_THREADS;  // entries per thread
  static_assert(PP * WP == NP && CC * G == CB, "tile split");
};

// The products of this wave's units, (pair w mod WP + WP i, column block
// w / WP + G j) for i < PP, j < CC: acc[i][j][t] (t < TILES) = row block
// t of pair i times column block j of Wreal * B, with Wreal the real form
// of F (or conj(F)).  The root of unity of a pair (A operand) is read once
// per k-step for all its column blocks, the B value once for all pairs.
template <int NT, bool CONJ>
__device__ __forceinline__ void dft_units(
    const double* B, const cx<double>* twl,
    dbl4 (&acc)[DftShape<NT>::PP][DftShape<NT>::CC][2]) {
  using SH = DftShape<NT>;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  int m[SH::PP], pr0[SH::PP], col[SH::CC];
#pragma unroll
  for (int i = 0; i < SH::PP; ++i) {
    const int p = wave % SH::WP + SH::WP * i;
    const int row0 = 16 * p + r;  // the lane's A row
    m[i] = row0 % NT;
    pr0[i] = row0 / NT;  // 1 only for the lower half of NT = 8
#pragma unroll
    for (int j = 0; j < SH::CC; ++j) {
      acc[i][j][0] = dbl4{0.0, 0.0, 0.0, 0.0};
      acc[i][j][1] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
  }
#pragma unroll
  for (int j = 0; j < SH::CC; ++j)
    col[j] = 16 * (wave / SH::WP + SH::G * j) + r;
#pragma unroll 2
  for (int ks = 0; ks < 2 * NT / 4; ++ks) {
    const int k = 4 * ks + q;
    const int l = k & (NT - 1);
    const int pc = k / NT;
    double b[SH::CC];
#pragma unroll
    for (int j = 0; j < SH::CC; ++j) b[j] = B[k * SH::LD + col[j]];
#pragma unroll
    for (int i = 0; i < SH::PP; ++i) {
      cx<double> w = twl[(m[i] * l) & (NT - 1)];
      if (CONJ) w.y = -w.y;
      // [[Re, -Im], [Im, Re]]: entry (pr, pc); the second row block of a
      // pair holds the imaginary parts (pr = 1)
      const double a0 = pr0[i] == pc ? w.x : (pr0[i] == 0 ? -w.y : w.y);
      const double a1 = pc == 1 ? w.x : w.y;
#pragma unroll
      for (int j = 0; j < SH::CC; ++j) {
        acc[i][j][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b[j],
                                                            acc[i][j][0], 0,
                                                            0, 0);
        if constexpr (SH::TILES == 2)
          acc[i][j][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              a1, b[j], acc[i][j][1], 0, 0, 0);
      }
    }
  }
}

// dft_units for an N-point transform (N <= NT, known at run time) placed
// in the NT-row tile: the complex matrix entry of row R and column K is
// w^{((R + roff) (K + koff)) mod N}, w = e^{+2 pi i/N} read from roots[N]
// (conjugated for CONJ).  The caller's offsets keep both factors
// non-negative (an index i - o of the unknown rows enters as i + N - o,
// the same exponent mod N); rows and columns outside the transform
// receive finite entries that a zero operand row or an ignored output
// masks.  Along a wave's k-steps the column index
// advances by 4, so each pair's exponent advances by 4 (R + roff) mod N
// and is kept reduced with one compare.
template <int NT, bool CONJ>
__device__ __forceinline__ void dft_units_n(
    const double* B, const cx<double>* roots, int N, int roff, int koff,
    dbl4 (&acc)[DftShape<NT>::PP][DftShape<NT>::CC][2]) {
  using SH = DftShape<NT>;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  int idx0[SH::PP], step[SH::PP], pr0[SH::PP], col[SH::CC];
#pragma unroll
  for (int i = 0; i < SH::PP; ++i) {
    const int p = wave % SH::WP + SH::WP * i;
    const int row0 = 16 * p + r;  // the lane's A row
    const int am = row0 % NT + roff;
    pr0[i] = row0 / NT;  // 1 only for the lower half of NT = 8
    idx0[i] = (am * (q + koff)) % N;
    step[i] = (4 * am) % N;
#pragma unroll
    for (int j = 0; j < SH::CC; ++j) {
      acc[i][j][0] = dbl4{0.0, 0.0, 0.0, 0.0};
      acc[i][j][1] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
  }
#pragma unroll
  for (int j = 0; j < SH::CC; ++j)
    col[j] = 16 * (wave / SH::WP + SH::G * j) + r;
  // the real (pc = 0) and imaginary (pc = 1) halves of the operand rows
#pragma unroll
  for (int pc = 0; pc < 2; ++pc) {
    int idx[SH::PP];
#pragma unroll
    for (int i = 0; i < SH::PP; ++i) idx[i] = idx0[i];
#pragma unroll 2
    for (int ks = 0; ks < NT / 4; ++ks) {
      const int k = pc * NT + 4 * ks + q;
      double b[SH::CC];
#pragma unroll
      for (int j = 0; j < SH::CC; ++j) b[j] = B[k * SH::LD + col[j]];
#pragma unroll
      for (int i = 0; i < SH::PP; ++i) {
        cx<double> w = roots[idx[i]];
        if (CONJ) w.y = -w.y;
        const double a0 = pr0[i] == pc ? w.x : (pr0[i] == 0 ? -w.y : w.y);
        const double a1 = pc == 1 ? w.x : w.y;
#pragma unroll
        for (int j = 0; j < SH::CC; ++j) {
          acc[i][j][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b[j],
                                                              acc[i][j][0], 0,
                                                              0, 0);
          if constexpr (SH::TILES == 2)
            acc[i][j][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                a1, b[j], acc[i][j][1], 0, 0, 0);
        }
        const int nx = idx[i] + step[i];
        idx[i] = nx >= N ? nx - N : nx;
      }
    }
  }
}

// Entry e of a unit's accumulators (e < 4 for NT >= 16: the complex entry
// of frequency/time row 16p + 4e + q, real part in acc[0][e], imaginary
// in acc[1][e]; e < 2 for NT = 8: row 4e + q, real acc[0][e], imaginary
// acc[0][e + 2]).
template <int NT>
struct DftEntry {
  static constexpr int N = NT >= 16 ? 4 : 2;
  __device__ static int row(int p, int e, int q) {
    return NT >= 16 ? 16 * p + 4 * e + q : 4 * e + q;
  }
  __device__ static cx<double> get(const dbl4 (&acc)[2], int e) {
    if constexpr (NT >= 16) return mk(acc[0][e], acc[1][e]);
    else return mk(acc[0][e], acc[0][e + 2]);
  }
};

// MODE: PB_ITERATE (residual, precondition, update) or PB_PRECOND.
template <int NT, int MODE, typename TN>
__device__ __forceinline__ void passb_dft_body(const PassBArgs& a, long lb,
                                               const TN* Nh, double* lds,
                                               double* red) {
  using SH = DftShape<NT>;
  constexpr int C = SH::C;
  constexpr int LD = SH::LD;
  using EN = DftEntry<NT>;
  double* B = lds;                                        // [2NT][LD]
  cx<double>* Ut = reinterpret_cast<cx<double>*>(lds + 2 * NT * LD);
  cx<double>* twl = Ut + NT * C;                          // [NT]
  cx<double>* lamc = twl + NT;                            // [NT]
  cx<double>* Ec = lamc + NT;                             // [C]
  double* gml = reinterpret_cast<double*>(Ec + C);        // [NT]
  const long Nk = a.Nk;
  const long k0 = lb * C;
  double nrm_r = 0.0, nrm_s = 0.0, nrm_u = 0.0;

  // tables: w^j = e^{+2 pi i j/NT} (conjugates of the e^{-2 pi i j/4096}
  // table), lambda_m, gamma_l, E of the tile's columns
  for (int j = threadIdx.x; j < NT; j += DENSE_THREADS) {
    twl[j] = conj(a.tw[j * (TW_N / NT)]);
    lamc[j] = a.lam[j];
    gml[j] = a.gam[j];
  }
  for (int c = threadIdx.x; c < C; c += DENSE_THREADS) {
    const long kap = k0 + c;
    Ec[c] = kap < Nk ? a.E[kap] : mk(0.0, 0.0);
  }
  // 1. rows of U into LDS (the residual needs u_{l-1}; the update u_l)
  if constexpr (MODE == PB_ITERATE) {
#pragma unroll
    for (int pp = 0; pp < SH::PER; ++pp) {
      const int e = threadIdx.x + pp * DENSE_THREADS;
      const int l = e / C, c = e % C;
      const long kap = k0 + c;
      Ut[e] = kap < Nk ? a.U[l * Nk + kap] : mk(0.0, 0.0);
    }
  }
  __syncthreads();
  // 2. gamma_l R_l as the real product operand
#pragma unroll
  for (int pp = 0; pp < SH::PER; ++pp) {
    const int e = threadIdx.x + pp * DENSE_THREADS;
    const int l = e / C, c = e % C;
    const long kap = k0 + c;
    const bool valid = kap < Nk;
    const int kl = static_cast<int>((valid ? kap : 0) % a.nh);
    const double pw = !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
    cx<double> r = mk(0.0, 0.0);
    if constexpr (MODE == PB_PRECOND) {
      if (valid) r = a.Rin[l * Nk + kap];
    } else {
      if (valid) {
        const cx<double> prev = l == 0 ? a.u0h[kap] : Ut[(l - 1) * C + c];
        r = cmul(prev, Ec[c]) - Ut[e];
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
    B[l * LD + c] = gml[l] * r.x;
    B[(NT + l) * LD + c] = gml[l] * r.y;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, q = lane >> 4;
  // 3. step (a) on MFMA, step (b) in registers
  dbl4 acc[SH::PP][SH::CC][2];
  dft_units<NT, false>(B, twl, acc);
  __syncthreads();  // every wave has read B: the X tile replaces it
#pragma unroll
  for (int i = 0; i < SH::PP; ++i) {
    const int p = wave % SH::WP + SH::WP * i;
#pragma unroll
    for (int j = 0; j < SH::CC; ++j) {
      const int c = 16 * (wave / SH::WP + SH::G * j) + r16;
#pragma unroll
      for (int e = 0; e < EN::N; ++e) {
        const int m = EN::row(p, e, q);
        const cx<double> z = cmul(lamc[m], Ec[c]);
        const double dr = 1.0 - z.x, di = -z.y;
        const double inv =
            1.0 / (static_cast<double>(NT) * (dr * dr + di * di));
        const cx<double> x =
            cmul(EN::get(acc[i][j], e), mk(dr * inv, -di * inv));
        B[m * LD + c] = x.x;
        B[(NT + m) * LD + c] = x.y;
      }
    }
  }
  __syncthreads();
  // 4. step (c) on MFMA, then 1/gamma_l and the update in registers
  dft_units<NT, true>(B, twl, acc);
#pragma unroll
  for (int i = 0; i < SH::PP; ++i) {
    const int p = wave % SH::WP + SH::WP * i;
#pragma unroll
    for (int j = 0; j < SH::CC; ++j) {
      const int c = 16 * (wave / SH::WP + SH::G * j) + r16;
      const long kap = k0 + c;
      const bool valid = kap < Nk;
      const int kl = static_cast<int>((valid ? kap : 0) % a.nh);
      const double pw =
          !valid ? 0.0 : ((kl == 0 || kl == a.nh - 1) ? 1.0 : 2.0);
#pragma unroll
      for (int e = 0; e < EN::N; ++e) {
        const int l = EN::row(p, e, q);
        const cx<double> sv = EN::get(acc[i][j], e) * (1.0 / gml[l]);
        nrm_s += pw * norm2(sv);
        if constexpr (MODE == PB_ITERATE) {
          const cx<double> un = Ut[l * C + c] + sv;
          nrm_u += pw * norm2(un);
          if (valid) a.U[l * Nk + kap] = un;
        } else {
          if (valid) a.Sout[l * Nk + kap] = sv;
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

template <int NT>
constexpr int dft_lds_doubles() {
  using SH = DftShape<NT>;
  // B, U tile, roots, lambda, E, gamma
  return 2 * NT * SH::LD + 2 * NT * SH::C + 2 * NT + 2 * NT + 2 * SH::C + NT;
}

template <int NT, int MODE, typename TN>
__global__ void __launch_bounds__(DENSE_THREADS)
    passb_dense_kernel(const PassBArgs* __restrict__ jobs,
                       const int* __restrict__ start, int njobs) {
  __shared__ double lds[dft_lds_doubles<NT>()];
  __shared__ double red[(DENSE_THREADS / 64) * 4];
  const int j = find_job(start, njobs);
  const PassBArgs a = jobs[j];
  const long lb = blockIdx.x - start[j];
  if constexpr (MODE == PB_ITERATE) {
    const int ph = job_phase(a.ctl);
    if (ph < 0) return;
    if (lb == 0 && threadIdx.x == 0) {
      a.ctl->pending = 1;
      a.ctl->zstart = 0;  // the next pass A computes again
    }
    if (a.Nh32 != nullptr && ph == PH_BULK)
      passb_dft_body<NT, MODE, float>(
          a, lb, static_cast<const float*>(a.Nh32), lds, red);
    else
      passb_dft_body<NT, MODE, double>(
          a, lb, static_cast<const double*>(a.Nh), lds, red);
  } else {
    passb_dft_body<NT, MODE, TN>(a, lb, static_cast<const TN*>(a.Nh), lds,
                                 red);
  }
}

template <int NT, int MODE, typename TN>
__global__ void __launch_bounds__(DENSE_THREADS)
    passb_dense_kernel1(PassBArgs a) {
  __shared__ double lds[dft_lds_doubles<NT>()];
  __shared__ double red[(DENSE_THREADS / 64) * 4];
  passb_dft_body<NT, MODE, TN>(a, blockIdx.x, static_cast<const TN*>(a.Nh),
                               lds, red);
}

}  // namespace expdiag
