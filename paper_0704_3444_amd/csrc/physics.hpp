// Per-site pieces of the method, shared by every kernel of the library.
//
//   chemical potential  Eq. (lgf) of Sec. IV, per mer, plus -kappa lap rho
//   force               Eq. (definef), either line
//   equilibrium         moments of Sec. III (second-order polynomial)
//   forcing term        moments Eqs. (ff1)-(ff3)
//   collision           Eq. (ssLB), BGK
//
// Populations live in "pull" storage: slot (sigma, i, r) holds the
// post-collision value f*_i computed at site r, so the population that sits
// at site r at the next step is the one stored at r - v_i.
//
// Layout in HBM (storage.hpp, BlockLayout): sites are grouped in blocks of
// 64 consecutive x on one row (row = y + ny z); a block stores the N*Q
// populations of its 64 sites as N*Q contiguous runs of 64 values.  A
// wavefront that owns one block reads and writes one contiguous region per
// step, so the N*Q population streams do not land on the same HBM channels
// at the same time (a plain structure of arrays puts them a power-of-two
// apart).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm {

constexpr int kMaxComp = 8;

// Scale of the shifted FP16 storage per component (unused by the other
// codecs); the references themselves are stored with the populations.
struct ShiftRef {
  float scale[kMaxComp];      // s^sigma, a power of two
  float inv_scale[kMaxComp];  // 1 / s^sigma
  float one, minus_one;       // 1 and -1, as run-time factors of the codec's FMAs (storage.hpp)
};

// Arithmetic parameters of one run, in the working precision T.
template <typename T>
struct Params {
  int n;          // number of components N
  int log_form;   // 1: A = -c rho grad(mu - ln(rho)/3); 0: A = -c (rho grad mu - grad(rho)/3)
  int nx, ny, nz;
  long long S;    // nx * ny * nz
  int nbx;        // 64-site blocks per row, ceil(nx / 64)
  int nq;         // populations per site, N * Q
  int walls;      // bit a: axis a closed by walls (split path only; 0 elsewhere)
  int pad_;
  T inv_tau;      // BGK rate 1/tau
  T cforce;       // c = w / tau = 1 - 1/(2 tau)
  T theta;        // temperature of the free energy
  T kappa;        // square-gradient coefficient
  T inv_m[kMaxComp];
  T chi[kMaxComp * kMaxComp];  // leading dimension kMaxComp, symmetric
  ShiftRef sh;
};

// Natural logarithm and reciprocal in the working precision.  FP32 uses the
// hardware v_log_f32 (log2, about 1 ulp) and v_rcp_f32 (1 ulp): each costs one
// instruction instead of a correctly rounded library sequence, and their
// error is far below the FP32 storage rounding that dominates that path.
// FP64 uses the correctly rounded library functions.
__device__ __forceinline__ float ln_(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ double ln_(double x) { return log(x); }
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }

// Fused multiply-add.  The library is compiled without automatic
// contraction, so every rounding is the one written here: each kernel that
// evaluates these functions gets the same bits whatever the code around it.
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Potential that the force differentiates, at one site:
//   mu^s = theta [ -1 + (1 + ln phi^s)/m^s - sum_t phi^t/m^t
//                  + sum_t chi^{st} phi^t - 1/2 sum_{t,t'} chi^{tt'} phi^t phi^t' ]
//          - kappa lap^s
//   h^s  = mu^s - ln(rho^s)/3   (log form)   or   mu^s   (expanded form)
// NC is the compile-time component count (n <= NC; entries >= n are ignored).
// EXACT: the caller is instantiated for n itself (n == NC), which removes
// the run-time guards and their branches; the arithmetic is the same.
template <typename T, int NC, bool EXACT = false>
__device__ __forceinline__ void site_potential(const Params<T>& p, const T (&rho)[NC],
                                               const T (&lap)[NC], T (&mu)[NC], T (&h)[NC]) {
  const int n = EXACT ? NC : p.n;
  T rt = T(0);
#pragma unroll
  for (int s = 0; s < NC; ++s)
    if (s < n) rt += rho[s];
  const T inv_rt = rcp_(rt);
  const T ln_rt = ln_(rt);
  T phi[NC];
  T sum_phi_m = T(0);
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    phi[s] = s < n ? rho[s] * inv_rt : T(0);
    sum_phi_m = fma_(phi[s], p.inv_m[s], sum_phi_m);
  }
  T lin[NC];
  T quad = T(0);
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    T acc = T(0);
#pragma unroll
    for (int t = 0; t < NC; ++t) acc = fma_(p.chi[s * kMaxComp + t], phi[t], acc);
    lin[s] = acc;
    quad = fma_(phi[s], acc, quad);
  }
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    if (s < n) {
      const T ln_rs = ln_(rho[s]);
      const T ln_phi = ln_rs - ln_rt;
      const T bulk = fma_(T(-0.5), quad, (fma_(T(1) + ln_phi, p.inv_m[s], T(-1)) - sum_phi_m) + lin[s]);
      mu[s] = fma_(p.theta, bulk, -(p.kappa * lap[s]));
      h[s] = p.log_form ? fma_(ln_rs, T(-1.0 / 3.0), mu[s]) : mu[s];
    } else {
      mu[s] = T(0);
      h[s] = T(0);
    }
  }
}

// Free-energy density psi of Eq. (lgf) at one site (bulk part only), used by
// the pressure diagnostic.
template <typename T, int NC>
__device__ __forceinline__ T site_psi(const Params<T>& p, const T (&rho)[NC]) {
  const int n = p.n;
  T rt = T(0);
#pragma unroll
  for (int s = 0; s < NC; ++s)
    if (s < n) rt += rho[s];
  T psi = T(0);
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    if (s < n) {
      const T phi = rho[s] / rt;
      const T num = rho[s] * p.inv_m[s];
      psi += p.theta * num * (ln_(phi) - T(1) / p.inv_m[s]);
#pragma unroll
      for (int t = 0; t < NC; ++t)
        if (t < n) psi += T(0.5) * p.theta * p.chi[s * kMaxComp + t] * rho[s] * (rho[t] / rt);
    }
  }
  return psi;
}

// BGK collision of one component at one site, Eq. (ssLB):
//   f*_i = f_i + (f^e_i - f_i)/tau + F_i = (1 - 1/tau) f_i + G_i,
//   G_i   = f^e_i / tau + F_i,
//   f^e_i = w_i rho [1 + 3 v.u + 9/2 (v.u)^2 - 3/2 u.u]      (barycentric u)
//   F_i   = w_i [3 v.A + 9 (v.A)(v.us) - 3 A.us]            (us = j / rho)
// Opposite velocities share the even parts of f^e and F and flip the odd
// ones, so each pair (i, opp(i)) forms G_e + G_o and G_e - G_o; products of
// the weight with per-site quantities are formed once per weight value.
// The zeroth moments of f^e and F (rho and 0) fix the rest population:
//   f*_0 = f_0 + sum_{i>0} (f_i - f*_i).
// Written this way the stored populations keep their exact sum up to the
// single rounding of f*_0: each difference f_i - f*_i is exact (the two
// values lie within a factor two of each other), whereas forming f^e_0 and
// F_0 separately lets biased roundings of the FP32 density sum drift the
// mass by ~1e-8 per step.
// v_i . (x, y, z) with the lattice's integer components folded in.
template <int LAT, typename T>
__device__ __forceinline__ T vdot(int i, T x, T y, T z) {
  using L = Lattice<LAT>;
  T r = T(0);
  bool any = false;
  if (L::cx(i)) { r = L::cx(i) > 0 ? x : -x; any = true; }
  if (L::cy(i)) { r = any ? (L::cy(i) > 0 ? r + y : r - y) : (L::cy(i) > 0 ? y : -y); any = true; }
  if (L::cz(i)) { r = any ? (L::cz(i) > 0 ? r + z : r - z) : (L::cz(i) > 0 ? z : -z); }
  return r;
}

template <int LAT, typename T>
__device__ __forceinline__ void collide(T (&f)[Lattice<LAT>::Q], T rho, T ux, T uy, T uz, T Ax,
                                        T Ay, T Az, T usx, T usy, T usz, T inv_tau) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  const T keep = T(1) - inv_tau;
  const T uu = L::D == 3 ? fma_(uz, uz, fma_(uy, uy, ux * ux)) : (L::D == 2 ? fma_(uy, uy, ux * ux) : ux * ux);
  const T Aus = L::D == 3 ? fma_(Az, usz, fma_(Ay, usy, Ax * usx)) : (L::D == 2 ? fma_(Ay, usy, Ax * usx) : Ax * usx);
  // the rate folded into the equilibrium's coefficients once per site:
  //   G_even = (rho w / tau) [1 - 3/2 u.u + 9/2 (v.u)^2] - 3 w A.us + 9 w (v.A)(v.us)
  //   G_odd  = (rho w / tau) 3 v.u + 3 w v.A
  const T t_base = inv_tau * fma_(T(-1.5), uu, T(1));
  const T t_sq = inv_tau * T(4.5), t_lin = inv_tau * T(3);
  T defect = T(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (L::opp(i) < i) continue;
    const int j = L::opp(i);
    // per weight value (the compiler forms these once per distinct w)
    const T wr = T(L::w(i)) * rho;
    const T a_sq = wr * t_sq, a_lin = wr * t_lin;
    const T a_0 = fma_(wr, t_base, T(-3.0 * L::w(i)) * Aus);
    const T vu = vdot<LAT, T>(i, ux, uy, uz);
    const T vA = vdot<LAT, T>(i, Ax, Ay, Az);
    const T vus = vdot<LAT, T>(i, usx, usy, usz);
    const T G_even = fma_(a_sq, vu * vu, fma_(T(9.0 * L::w(i)) * vA, vus, a_0));
    const T G_odd = fma_(a_lin, vu, T(3.0 * L::w(i)) * vA);
    const T post_i = fma_(keep, f[i], G_even + G_odd);
    const T post_j = fma_(keep, f[j], G_even - G_odd);
    defect += f[i] - post_i;
    defect += f[j] - post_j;
    f[i] = post_i;
    f[j] = post_j;
  }
  f[0] = f[0] + defect;
}

// Stencils, written once so that every kernel forms them in the same order.
// `g(i)` returns the field at r + v_i.
//   lap g   = 6 sum_{i>0} w_i (g(r + v_i) - g(r)) = 6 sum_{i>0} w_i g(r + v_i) - 6 W g(r),
//             W = sum_{i>0} w_i = 1 - w_0 (formed the second way: one FMA per neighbour)
//   grad g  = 3 sum_{i>0} w_i v_i g(r + v_i)
template <int LAT, typename T, typename G>
__device__ __forceinline__ T lattice_laplacian(const G& g, T g0) {
  using L = Lattice<LAT>;
  constexpr double kW = 1.0 - L::w(0);
  T acc = T(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) acc = fma_(T(L::w(i)), g(i), acc);
  return fma_(T(6), acc, T(-6.0 * kW) * g0);
}

// sum_{i>0} w_i v_i g(r + v_i): one third of the gradient stencil.
template <int LAT, typename T, typename G>
__device__ __forceinline__ void lattice_wsum(const G& g, T& sx, T& sy, T& sz) {
  using L = Lattice<LAT>;
  sx = sy = sz = T(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    const T v = g(i);
    if (L::cx(i)) sx = fma_(T(L::cx(i) * L::w(i)), v, sx);
    if (L::cy(i)) sy = fma_(T(L::cy(i) * L::w(i)), v, sy);
    if (L::cz(i)) sz = fma_(T(L::cz(i) * L::w(i)), v, sz);
  }
}

// Force density A = rho^s a^s of Eq. (definef), c = 1 - 1/(2 tau):
//   log form:      A = -c rho grad h,                 h = mu - ln(rho)/3
//   expanded form: A = -c (rho grad h - grad(rho)/3), h = mu
// `h(i)` and `r(i)` give the potential and the density at r + v_i.
template <int LAT, typename T, typename GH, typename GR>
__device__ __forceinline__ void lattice_force(const GH& h, const GR& r, T rho_s, const Params<T>& p,
                                              T& Ax, T& Ay, T& Az) {
  T hx, hy, hz;
  lattice_wsum<LAT, T>(h, hx, hy, hz);
  T qx = T(0), qy = T(0), qz = T(0);
  if (!p.log_form) lattice_wsum<LAT, T>(r, qx, qy, qz);
  Ax = -p.cforce * fma_(rho_s, T(3) * hx, -qx);
  Ay = -p.cforce * fma_(rho_s, T(3) * hy, -qy);
  Az = -p.cforce * fma_(rho_s, T(3) * hz, -qz);
}

constexpr int kBlockX = 64;

// Periodic neighbour coordinate: x + d with d in {-1, 0, 1}.
__device__ __forceinline__ int wrap_add(int x, int d, int n) {
  int y = x + d;
  y = y < 0 ? y + n : y;
  return y >= n ? y - n : y;
}

}  // namespace lbm
