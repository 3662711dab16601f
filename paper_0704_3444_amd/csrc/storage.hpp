// How a copy of the populations is held in HBM, and how a kernel turns a
// stored slot into a population value and back.
//
//   StoreF64, StoreF32  every population in the working precision T.
//   StoreF16S           per site and component, an FP16 reference h, the
//                       moving populations (i > 0) as FP16 deviations d_i
//                       from the shifted equilibrium w_i (36 h s) of that
//                       reference, in units of s^sigma (a power of two), and
//                       the rest slot (i = 0) as an FP32 ledger.  All
//                       arithmetic stays in FP32.
//
// Shifted codec.  A slot written at site r decodes, wherever it is read, with
// the reference of r:  f = s (k_i h(r) + d),  k_i = 36 w_i  (an integer: 16,
// 4, 1 on D2Q9; 12, 2, 1 on D3Q19; 24, 6 on D1Q3; sum_i k_i = 36).  The
// collision at r sets h(r) = fl16(rho(r) / (36 s)), so the reference follows
// the site's own density and the deviations stay small where one component is
// scarce (a reference shared by a region puts the scarce phase of that region
// far from it, and FP16's 11 bits then round its populations coarsely).
//
// Ledger.  Every FP16 number is a multiple of 2^-24, and so are k_i h and the
// rest slot by construction.  A sum of such numbers is exact in FP32 while its
// partial sums stay below 1 in magnitude.  The pulled populations of a site,
// in units of s,  u_i = k_i h(src_i) + d_i  (u_0 = k_0 h(r) + rest slot),
// are therefore exact, and so is their sum  T = rho / s.  The collision writes
// the new reference h', the moving deviations d*_i = fl16(f*_i / s - k_i h')
// and, in the rest slot,  T - 36 h' - sum_{i>0} d*_i:  the stored total stays
// T exactly, so every collision keeps the component mass exactly, whatever
// FP16 rounded, and streaming moves stored values unchanged.  s is twice the
// smallest power of two not below max rho0^sigma, so the sums stay exact
// until a density doubles that maximum (beyond, they round at 2^-23 s, still
// far below FP16's steps).
//
// Block layout (all codecs): sites are grouped in blocks of 64 consecutive
// x on one row (row = y + ny z).  A block stores, for each component, the
// rest run (64 Rest values), the Q - 1 moving runs (64 Move values each) in
// the run order run_slot(i), and for the shifted codec one reference run (64
// FP16 h values) after the first ref_pos - 1 runs.  On D2Q9 the runs are
// grouped by the y component of the velocity, v_y = 0 (i = 0, 1, 3, and the
// references), +1 (2, 5, 6), -1 (4, 7, 8): the populations that one row pulls
// from each of its three source rows are then one contiguous piece of that
// row's block per component.  Other lattices keep the order of the velocity
// table, with the references after the rest run.
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
  static constexpr uint32_t kRef = 0;  // bytes of the reference per site
  static constexpr int kId = 0;
};
struct StoreF32 {
  using T = float;
  using Rest = float;
  using Move = float;
  static constexpr bool kShift = false;
  static constexpr uint32_t kRef = 0;
  static constexpr int kId = 1;
};
struct StoreF16S {
  using T = float;
  using Rest = float;
  using Move = _Float16;
  static constexpr bool kShift = true;
  static constexpr uint32_t kRef = 2;
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

// Run position before which the reference run sits (shifted codec): after
// the v_y = 0 group on D2Q9, after the rest run elsewhere.
template <int Q>
__host__ __device__ constexpr int ref_pos() {
  return Q == 9 ? 3 : 1;
}

template <class S, int Q>
struct BlockLayout {
  static constexpr uint32_t kRest = sizeof(typename S::Rest);
  static constexpr uint32_t kMove = sizeof(typename S::Move);
  static constexpr uint32_t kRef = S::kRef;
  // bytes of one component in one block
  static constexpr uint32_t kComp = kBlockX * (kRest + kRef + (Q - 1) * kMove);
  // offset of the run of population i of component c inside a block
  static constexpr uint32_t run(int c, int i) {
    const int j = run_slot<Q>(i);
    return uint32_t(c) * kComp +
           (i == 0 ? 0u : kBlockX * (kRest + uint32_t(j - 1) * kMove + (j >= ref_pos<Q>() ? kRef : 0u)));
  }
  // offset of the reference run of component c inside a block
  static constexpr uint32_t ref(int c) {
    return uint32_t(c) * kComp + kBlockX * (kRest + uint32_t(ref_pos<Q>() - 1) * kMove);
  }
  // offset of site x within its run
  static constexpr uint32_t in_run(int i, int x) { return uint32_t(x & (kBlockX - 1)) * (i == 0 ? kRest : kMove); }
  static constexpr uint32_t in_ref(int x) { return uint32_t(x & (kBlockX - 1)) * kRef; }
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

// Byte offset of the reference of component c at site (x, row) (shifted codec).
template <class S, int Q>
__device__ __forceinline__ uint64_t ref_byte(int n, int nbx, int c, int x, long long row) {
  return block_byte<S, Q>(n, nbx, x, row) + BlockLayout<S, Q>::ref(c) + BlockLayout<S, Q>::in_ref(x);
}

// Raw slot value converted to the working precision (exact for every codec).
template <class S>
__device__ __forceinline__ typename S::T load_slot(const void* base, uint64_t off, int i) {
  const char* b = static_cast<const char*>(base) + off;
  if (i == 0) return typename S::T(*reinterpret_cast<const typename S::Rest*>(b));
  return typename S::T(*reinterpret_cast<const typename S::Move*>(b));
}

// FP16 value (a moving slot or a reference of the shifted codec) and FP32
// rest slot at a byte offset.
__device__ __forceinline__ _Float16 load_half(const void* base, uint64_t off) {
  return *reinterpret_cast<const _Float16*>(static_cast<const char*>(base) + off);
}
__device__ __forceinline__ float load_f32(const void* base, uint64_t off) {
  return *reinterpret_cast<const float*>(static_cast<const char*>(base) + off);
}

// k_i = 36 w_i, the multiple of the reference in the shifted equilibrium of
// direction i (an integer for every velocity set here).
template <int LAT>
__host__ __device__ constexpr float ref_weight(int i) {
  return float(int(36.0 * Lattice<LAT>::w(i) + 0.5));
}

template <int LAT>
constexpr bool ref_weights_exact() {
  int sum = 0;
  for (int i = 0; i < Lattice<LAT>::Q; ++i) {
    const double k = 36.0 * Lattice<LAT>::w(i);
    if (k - double(ref_weight<LAT>(i)) > 1e-12 || double(ref_weight<LAT>(i)) - k > 1e-12) return false;
    sum += int(ref_weight<LAT>(i));
  }
  return sum == 36;
}
static_assert(ref_weights_exact<1>() && ref_weights_exact<2>() && ref_weights_exact<3>(), "36 w_i integral");

// a h + d with h and d FP16, rounded once (for the codec's values the result
// is exact).  Written as an FMA of the converted operands, which the compiler
// turns into one v_fma_mix_f32 (converting the FP16 operands itself) unless
// it can simplify the FMA: a factor of 1 or -1 would become an add, with two
// separate conversions.  Such factors therefore come from the run's
// parameters (ShiftRef::one, ShiftRef::minus_one), which the compiler cannot
// fold.
__device__ __forceinline__ float mix_fma(float a, _Float16 h, _Float16 d) {
  return __builtin_fmaf(a, float(h), float(d));
}

// Take pulled slot i (raw value in the working precision) into the
// population value f and the site's running sum, in direction order (plain
// codecs).
template <class S, int LAT>
__device__ __forceinline__ void take_slot(int i, typename S::T raw, typename S::T& sum, typename S::T& f) {
  static_assert(!S::kShift, "plain codecs");
  sum = i == 0 ? raw : sum + raw;
  f = raw;
}

// The same for the shifted codec: slot i holds the FP16 deviation d (i > 0)
// or the FP32 rest value (i == 0), written by the site whose reference is h.
// Sums u_i = k_i h + d in units of s (exact) and returns f = s u_i.  `one`
// is ShiftRef::one (1.0, the factor of the directions with k_i = 1).
template <int LAT>
__device__ __forceinline__ void take_shifted(int i, _Float16 d, float rest, _Float16 h, float scale, float one,
                                             float& sum, float& f) {
  const float k = ref_weight<LAT>(i) == 1.0f ? one : ref_weight<LAT>(i);
  const float u = i == 0 ? __builtin_fmaf(k, float(h), rest) : mix_fma(k, h, d);
  sum = i == 0 ? u : sum + u;
  f = u * scale;
}

// The same population exactly in FP64 (k_i h + d is exact in FP32 already;
// the power-of-two scale keeps it exact).
template <class S, int LAT>
__device__ __forceinline__ double take_exact(int i, typename S::T raw, float h, float scale) {
  if constexpr (S::kShift) {
    return double(scale) * (double(ref_weight<LAT>(i)) * double(h) + double(raw));
  } else {
    return double(raw);
  }
}

// Component density of one site from the running sum of take_slot: the
// direction-order sum itself (plain codecs) or s T (shifted codec, exact).
template <class S>
__device__ __forceinline__ typename S::T site_density(typename S::T sum, float scale) {
  if constexpr (S::kShift) {
    return sum * scale;
  } else {
    return sum;
  }
}

// New reference of a site from its pulled total T = rho / s (shifted codec).
__device__ __forceinline__ _Float16 new_ref(float sum) {
#pragma clang fp contract(off)
  return _Float16(sum * (1.0f / 36.0f));
}

// Moving deviation d*_i of a post-collision value against the site's new
// reference h' (shifted codec): fl16(f*_i / s - k_i h'), with f*_i / s exact.
template <int LAT>
__device__ __forceinline__ _Float16 encode_move(int i, float post, float inv_scale, float h) {
  return _Float16(__builtin_fmaf(post, inv_scale, -(ref_weight<LAT>(i) * h)));
}

// Rest slot that keeps the stored total at T: T - 36 h' - sum_{i>0} d*_i,
// each step exact.  `d` holds the stored moving deviations (index 0 unused);
// each subtraction is an FMA of the FP16 value by `minus_one`
// (ShiftRef::minus_one, -1.0), one v_fma_mix_f32.
template <int Q>
__device__ __forceinline__ float ledger_rest(float sum, float h, const _Float16 (&d)[Q], float minus_one) {
#pragma clang fp contract(off)
  float rest = sum - 36.0f * h;
#pragma unroll
  for (int i = 1; i < Q; ++i) rest = __builtin_fmaf(float(d[i]), minus_one, rest);
  return rest;
}

}  // namespace lbm
