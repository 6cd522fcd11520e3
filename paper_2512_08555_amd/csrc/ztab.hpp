// Layout of the later-stage twiddle tables of the wave-per-line transforms
// (length M = 64 E), shared by the twiddle-table builder (which stores them
// after each axis table) and the kernels (which copy them into LDS):
//   t2[l1 (E+1) + m1]       = w_M^(E l1 m1),  l1 < A, m1 <= E  (forward stage 2)
//   ta[(n0-1) (M/A) + a]    = w_M^(n0 a),     0 < n0 < A, a < M/A  (inverse stage A)
//   tb[b (E+1) + e]         = w_M^(A e b),    b < E, e <= E    (inverse stage B)
// with w_M = exp(-2 pi i / M) and A = 64 / E.  Rows of E+1 entries put the
// lane groups that read different rows of t2 and tb in different LDS banks.
#pragma once

namespace ups {

template <int E>
struct ZTab {
  static constexpr int M = 64 * E, A = 64 / E;
  static constexpr int n2 = A * (E + 1), na = (A - 1) * (M / A), nb = E * (E + 1);
  static constexpr int o2 = 0, oa = n2, ob = n2 + na, total = n2 + na + nb;
};

// Exponent m of entry i (the entry is w_M^m, 0 <= m < M).
template <int E>
constexpr long long ztab_exponent(int i) {
  using Z = ZTab<E>;
  constexpr int M = Z::M, A = Z::A;
  if (i < Z::oa) return (long long)E * (i / (E + 1)) * (i % (E + 1)) % M;
  if (i < Z::ob) {
    const int j = i - Z::oa;
    return (long long)(j / (M / A) + 1) * (j % (M / A));  // n0 a < M
  }
  const int j = i - Z::ob;
  return (long long)A * (j / (E + 1)) * (j % (E + 1)) % M;
}

// Entries of the tables for a transform of length M (0 where the
// wave-per-line kernels do not exist).
inline int ztab_entries(int M) {
  switch (M) {
    case 512: return ZTab<8>::total;
    case 1024: return ZTab<16>::total;
    case 2048: return ZTab<32>::total;
    case 4096: return ZTab<64>::total;
    default: return 0;
  }
}

}  // namespace ups
