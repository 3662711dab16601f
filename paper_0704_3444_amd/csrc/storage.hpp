// How a copy of the populations is held in HBM, and how a kernel turns a
// stored slot into a population value and back.
//
//   StoreF64, StoreF32  every population in the working precision T.
//   StoreF16S           moving populations (i > 0) as FP16 deviations from
//                       the shifted equilibrium w_i rbar^sigma of the mean
//                       density, scaled by 1/s^sigma (s a power of two);
//                       the rest slot (i = 0) as an FP32 ledger.  All
//                       arithmetic stays in FP32.
//
// Ledger of StoreF16S.  In units of s, every FP16 value is a multiple of
// 2^-24, and so is the rest slot by construction.  A sum of such numbers is
// exact in FP32 while its partial sums stay below 1 in magnitude.  A site
// therefore holds the exact total deviation
//     L = d_0 + sum_{i>0} d_i,     rho = sum_i C_i + s L,   C_i = w_i rbar,
// and after the collision writes its moving deviations d*_i (each rounded to
// FP16) and d*_0 = L - sum_{i>0} d*_i.  The rest slot absorbs all FP16
// rounding, so every collision keeps the component mass exactly, and
// streaming moves stored values unchanged.  s is the smallest power of two
// not below max rho0^sigma, so |L| < 1 holds until a density exceeds
// rbar + s (beyond that the sums round at 2^-23 s, still far below FP16).
//
// Block layout (all codecs): sites are grouped in blocks of 64 consecutive
// x on one row (row = y + ny z).  A block stores, for each component, the
// rest run (64 Rest values) followed by the Q - 1 moving runs (64 Move
// values each), in the run order run_slot(i).  On D2Q9 the runs are grouped
// by the y component of the velocity, v_y = 0 (i = 0, 1, 3), +1 (2, 5, 6),
// -1 (4, 7, 8): the populations that one row pulls from each of its three
// source rows are then one contiguous piece of that row's block per
// component.  Other lattices keep the order of the velocity table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"
#include "physics.hpp"

namespace lbm {

struct StoreF64 {
  using T = double;
  using Rest = double;
  using Move = double;
  static constexpr bool kShift = false;
  static constexpr int kId = 0;
};
struct StoreF32 {
  using T = float;
  using Rest = float;
  using Move = float;
  static constexpr bool kShift = false;
  static constexpr int kId = 1;
};
struct StoreF16S {
  using T = float;
  using Rest = float;
  using Move = _Float16;
  static constexpr bool kShift = true;
  static constexpr int kId = 2;
};

// Position of velocity i in a component's run order.
template <int Q>
__host__ __device__ constexpr int run_slot(int i) {
  if constexpr (Q == 9) {
    constexpr int slot[9] = {0, 1, 3, 2, 6, 4, 5, 7, 8};  // 0 1 3 | 2 5 6 | 4 7 8
    return slot[i];
  } else {
    return i;
  }
}

template <class S, int Q>
struct BlockLayout {
  static constexpr uint32_t kRest = sizeof(typename S::Rest);
  static constexpr uint32_t kMove = sizeof(typename S::Move);
  // bytes of one component in one block
  static constexpr uint32_t kComp = kBlockX * (kRest + (Q - 1) * kMove);
  // offset of the run of population i of component c inside a block
  static constexpr uint32_t run(int c, int i) {
    return uint32_t(c) * kComp + (i == 0 ? 0u : kBlockX * (kRest + uint32_t(run_slot<Q>(i) - 1) * kMove));
  }
  // offset of site x within its run
  static constexpr uint32_t in_run(int i, int x) { return uint32_t(x & (kBlockX - 1)) * (i == 0 ? kRest : kMove); }
};

// Byte offset of the block that holds site (x, row), 64-bit.
template <class S, int Q>
__device__ __forceinline__ uint64_t block_byte(int n, int nbx, int x, long long row) {
  return (uint64_t(row) * uint64_t(nbx) + uint64_t(x >> 6)) * uint64_t(n) * BlockLayout<S, Q>::kComp;
}

// Byte offset of population i of component c at site (x, row), 64-bit.
template <class S, int Q>
__device__ __forceinline__ uint64_t pop_byte(int n, int nbx, int c, int i, int x, long long row) {
  return block_byte<S, Q>(n, nbx, x, row) + BlockLayout<S, Q>::run(c, i) + BlockLayout<S, Q>::in_run(i, x);
}

// Raw slot value converted to the working precision (exact for every codec).
template <class S>
__device__ __forceinline__ typename S::T load_slot(const void* base, uint64_t off, int i) {
  const char* b = static_cast<const char*>(base) + off;
  if (i == 0) return typename S::T(*reinterpret_cast<const typename S::Rest*>(b));
  return typename S::T(*reinterpret_cast<const typename S::Move*>(b));
}

// Shifted equilibrium C_i = w_i rbar^sigma in FP32 (one rounding).
template <int LAT>
__device__ __forceinline__ float shift_ref(const ShiftRef& r, int c, int i) {
#pragma clang fp contract(off)
  return float(Lattice<LAT>::w(i)) * r.rbar[c];
}

// Population value from a raw slot value in the working precision: for the
// shifted codec, f = C_i + s d (one FP32 rounding).
template <class S, int LAT>
__device__ __forceinline__ typename S::T decode(const ShiftRef& r, int c, int i, typename S::T raw) {
  if constexpr (S::kShift) {
    return __builtin_fmaf(raw, r.scale[c], shift_ref<LAT>(r, c, i));
  } else {
    return raw;
  }
}

// The same value, exactly, in FP64 (C_i is an FP32 number and s d has at
// most 24 significant bits, so the sum needs no rounding in FP64).
template <class S, int LAT>
__device__ __forceinline__ double decode_exact(const ShiftRef& r, int c, int i, typename S::T raw) {
  if constexpr (S::kShift) {
    return double(shift_ref<LAT>(r, c, i)) + double(raw) * double(r.scale[c]);
  } else {
    return double(raw);
  }
}

// Component density of one site from its decoded populations (plain codecs:
// the sum in direction order) or from its ledger (shifted codec).
template <class S, int Q>
__device__ __forceinline__ typename S::T site_density(const ShiftRef& r, int c, const typename S::T (&f)[Q],
                                                      typename S::T ledger) {
  using T = typename S::T;
  if constexpr (S::kShift) {
    return __builtin_fmaf(ledger, r.scale[c], r.csum[c]);
  } else {
    T acc = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) acc += f[i];
    return acc;
  }
}

// Moving deviation d*_i of a post-collision value (shifted codec).
template <int LAT>
__device__ __forceinline__ _Float16 encode_move(const ShiftRef& r, int c, int i, float post) {
#pragma clang fp contract(off)
  return _Float16((post - shift_ref<LAT>(r, c, i)) * r.inv_scale[c]);
}

}  // namespace lbm
