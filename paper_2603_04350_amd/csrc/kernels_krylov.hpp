// Krylov-vector kernels for GMRES on spectral space-time vectors.
#pragma once
#include "cx.hpp"

namespace expdiag {

constexpr int KRY_THREADS = 256;
constexpr int KRY_PER_THREAD = 4;

inline long krylov_blocks(long n) {
  const long per = static_cast<long>(KRY_THREADS) * KRY_PER_THREAD;
  long b = (n + per - 1) / per;
  return b < 1 ? 1 : b;
}

}  // namespace expdiag
