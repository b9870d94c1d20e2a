// Integer velocity sets of the on-lattice quadratures, as compile-time tables.
//
// The lattice ES-BGK model (Sec. 2.2) evaluates the distribution at the
// abscissae c_alpha = r e_alpha of a Gauss-Hermite quadrature. On-lattice
// streaming needs integer e_alpha; the two sets used here are D2Q37 (exact to
// degree 9, carries the N = 4 expansion the paper uses) and D3Q39 (exact to
// degree 7, carries N = 3). Only the integer vectors are compile-time; the
// scale r and the weights are derived on the host at start-up (tables.cpp)
// and read by the kernels from device memory.
//
// Velocity order (shared with the population I/O of the C ABI): index 0 is
// the rest velocity, indices 1..P the vectors whose first non-zero component
// is positive, sorted by |e|^2 and then by descending tuple order, and index
// alpha + P holds -e_alpha. The kernels exploit the (alpha, alpha + P) pairing
// to split every polynomial in e into its even and odd parts.
#pragma once

namespace esbgk {

struct D2Q37 {
  static constexpr int D = 2;
  static constexpr int Q = 37;
  static constexpr int P = 18;   // number of (e, -e) pairs
  static constexpr int N = 4;    // Hermite order carried
  // representatives e_1..e_P (the opposites follow at +P)
  static constexpr int E[P][3] = {
      {1, 0, 0},  {0, 1, 0},                          // |e|^2 = 1
      {1, 1, 0},  {1, -1, 0},                         // 2
      {2, 0, 0},  {0, 2, 0},                          // 4
      {2, 1, 0},  {2, -1, 0}, {1, 2, 0}, {1, -2, 0},  // 5
      {2, 2, 0},  {2, -2, 0},                         // 8
      {3, 0, 0},  {0, 3, 0},                          // 9
      {3, 1, 0},  {3, -1, 0}, {1, 3, 0}, {1, -3, 0},  // 10
  };
};

struct D3Q39 {
  static constexpr int D = 3;
  static constexpr int Q = 39;
  static constexpr int P = 19;
  static constexpr int N = 3;
  static constexpr int E[P][3] = {
      {1, 0, 0},  {0, 1, 0},  {0, 0, 1},                                  // 1
      {1, 1, 1},  {1, 1, -1}, {1, -1, 1}, {1, -1, -1},                    // 3
      {2, 0, 0},  {0, 2, 0},  {0, 0, 2},                                  // 4
      {2, 2, 0},  {2, 0, 2},  {2, 0, -2}, {2, -2, 0}, {0, 2, 2}, {0, 2, -2},  // 8
      {3, 0, 0},  {0, 3, 0},  {0, 0, 3},                                  // 9
  };
};

// Component a of velocity alpha (0 <= alpha < Q), including the opposites.
template <class L>
__host__ __device__ constexpr int ecomp(int alpha, int a) {
  return alpha == 0 ? 0 : (alpha <= L::P ? L::E[alpha - 1][a] : -L::E[alpha - 1 - L::P][a]);
}

// The velocity -e_alpha.
template <class L>
__host__ __device__ constexpr int opposite(int alpha) {
  return alpha == 0 ? 0 : (alpha <= L::P ? alpha + L::P : alpha - L::P);
}

// The velocity whose last component (the wall normal) is that of alpha
// negated and whose other components are alpha's: the specular image at a
// wall across the last axis.
template <class L>
__host__ __device__ constexpr int mirror_search(int alpha) {
  for (int b = 0; b < L::Q; ++b) {
    bool same = ecomp<L>(b, L::D - 1) == -ecomp<L>(alpha, L::D - 1);
    for (int k = 0; k < L::D - 1; ++k) same = same && ecomp<L>(b, k) == ecomp<L>(alpha, k);
    if (same) return b;
  }
  return -1;
}

// The images of all velocities, as a constexpr variable: evaluated by the
// compiler, so that a kernel indexes a constant table (or, at an unrolled
// index, uses the constant) instead of running the search.
template <class L>
struct MirrorTable {
  int m[L::Q];
  constexpr MirrorTable() : m{} {
    for (int a = 0; a < L::Q; ++a) m[a] = mirror_search<L>(a);
  }
};
template <class L>
inline constexpr MirrorTable<L> mirror_table{};

template <class L>
__host__ __device__ constexpr int mirror(int alpha) {
  return mirror_table<L>.m[alpha];
}

template <class L>
constexpr bool mirror_is_an_involution() {
  for (int a = 0; a < L::Q; ++a)
    if (mirror<L>(a) < 0 || mirror<L>(mirror<L>(a)) != a) return false;
  return true;
}
static_assert(mirror_is_an_involution<D2Q37>() && mirror_is_an_involution<D3Q39>(),
              "every velocity needs a mirror image in the set");

}  // namespace esbgk
