// Velocity sets for the device code.  D1Q3 is the set of Sec. IV; D2Q9 and
// D3Q19 are the standard second-order sets (sum_i w_i v_i v_i = I/3, fourth
// moment isotropic).  Every table is a constexpr function so that fully
// unrolled loops fold each velocity component and weight into an immediate;
// opp(i) is the index of -v_i.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

template <int LAT>
struct Lattice;

template <>
struct Lattice<1> {  // D1Q3
  static constexpr int Q = 3, D = 1;
  __host__ __device__ static constexpr int cx(int i) { return i == 1 ? 1 : (i == 2 ? -1 : 0); }
  __host__ __device__ static constexpr int cy(int) { return 0; }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr double w(int i) { return i == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
  __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : 3 - i; }
};

template <>
struct Lattice<2> {  // D2Q9: rest, 4 axis, 4 diagonal
  static constexpr int Q = 9, D = 2;
  __host__ __device__ static constexpr int cx(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  __host__ __device__ static constexpr int opp(int i) {
    return i == 0 ? 0 : (i == 1 || i == 2 || i == 5 || i == 6 ? i + 2 : i - 2);
  }
};

template <>
struct Lattice<3> {  // D3Q19: rest, 6 axis, 12 edge
  static constexpr int Q = 19, D = 3;
  __host__ __device__ static constexpr int cx(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : ((i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : ((i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int i) {
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : ((i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0);
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : (i % 2 ? i + 1 : i - 1); }
};

// Compile-time checks of the tables: weights sum to one, opp(i) is -v_i.
template <typename L>
constexpr bool tables_consistent() {
  double ws = 0.0;
  for (int i = 0; i < L::Q; ++i) {
    ws += L::w(i);
    const int j = L::opp(i);
    if (L::cx(j) != -L::cx(i) || L::cy(j) != -L::cy(i) || L::cz(j) != -L::cz(i)) return false;
    if (L::w(j) != L::w(i)) return false;
  }
  return ws > 1.0 - 1e-15 && ws < 1.0 + 1e-15;
}
static_assert(tables_consistent<Lattice<1>>(), "D1Q3 table");
static_assert(tables_consistent<Lattice<2>>(), "D2Q9 table");
static_assert(tables_consistent<Lattice<3>>(), "D3Q19 table");

}  // namespace lbm
