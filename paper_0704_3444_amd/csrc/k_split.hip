// Generic kernels for every lattice and precision.
//
// The split step runs three kernels: k_density (rho^sigma), k_potential
// (mu^sigma and the potential the force differentiates) and k_collide
// (force, equilibrium, forcing term, BGK, and the write that streams by
// pull; for N <= 4 the component count is a template parameter of the
// potential and the collision).  It is the path for D1Q3 and D3Q19 and the cross-check of the
// fused D2Q9 kernel.  The same kernels, instantiated in FP64, produce the
// observables of lb_moments.  It is also the path that takes walls (a
// closed axis: bounce-back in the pull, mirrored layers in the stencils).
// k_diag/k_diag_final form the FP64 mass and
// momentum sums and the density health flag with a fixed reduction order.
// Every kernel is templated on the storage codec S (storage.hpp): T is its
// working precision; stored slots are decoded on load and encoded on store.
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"
#include "physics.hpp"
#include "storage.hpp"

namespace lbm {

constexpr int kBlock = 256;

struct SiteCoord {
  int x, y, z;
};

template <typename T>
__device__ __forceinline__ SiteCoord coord_of(long long s, const Params<T>& p) {
  SiteCoord c;
  c.x = int(s % p.nx);
  long long r = s / p.nx;
  c.y = int(r % p.ny);
  c.z = int(r / p.ny);
  return c;
}

template <typename T>
__device__ __forceinline__ long long site_of(int x, int y, int z, const Params<T>& p) {
  return (long long)x + (long long)p.nx * ((long long)y + (long long)p.ny * z);
}

// Coordinate x + d (|d| <= 1) along an axis of n layers: periodic, or, on
// an axis closed by walls, the mirror image of the layer next to the wall
// when x + d lies beyond it (zero normal gradient of the stencils' fields).
__device__ __forceinline__ int axis_step(int x, int d, int n, bool wall) {
  const int y = x + d;
  if (wall) return y < 0 ? -1 - y : (y >= n ? 2 * n - 1 - y : y);
  return wrap_add(x, d, n);
}

// Site r + sign * v_i for the stencils.
template <int LAT, typename T>
__device__ __forceinline__ long long neighbour(const SiteCoord& c, int i, int sign, const Params<T>& p) {
  using L = Lattice<LAT>;
  return site_of(axis_step(c.x, sign * L::cx(i), p.nx, p.walls & 1), axis_step(c.y, sign * L::cy(i), p.ny, p.walls & 2),
                 axis_step(c.z, sign * L::cz(i), p.nz, p.walls & 4), p);
}

// True when site c + sign * v_i lies beyond a wall.
template <int LAT, typename T>
__device__ __forceinline__ bool beyond_wall(const SiteCoord& c, int i, int sign, const Params<T>& p) {
  using L = Lattice<LAT>;
  const int x = c.x + sign * L::cx(i), y = c.y + sign * L::cy(i), z = c.z + sign * L::cz(i);
  return ((p.walls & 1) && (x < 0 || x >= p.nx)) || ((p.walls & 2) && (y < 0 || y >= p.ny)) ||
         ((p.walls & 4) && (z < 0 || z >= p.nz));
}

// Site that a population leaving c with velocity v_i reaches in one step:
// c + v_i, or c itself when a wall lies between (half-way bounce-back
// returns it there reversed).
template <int LAT, typename T>
__device__ __forceinline__ long long stream_target(const SiteCoord& c, int i, const Params<T>& p) {
  return beyond_wall<LAT>(c, i, +1, p) ? site_of(c.x, c.y, c.z, p) : neighbour<LAT>(c, i, +1, p);
}

// The slot pulled into site c along v_i: slot i of the site r - v_i, or,
// across a wall, slot -v_i of r itself (bounce-back).
struct SlotAt {
  int x;
  long long row;
  int i;
};

template <int LAT, typename T>
__device__ __forceinline__ SlotAt pull_slot(const SiteCoord& c, int i, const Params<T>& p) {
  using L = Lattice<LAT>;
  if (beyond_wall<LAT>(c, i, -1, p)) return {c.x, (long long)c.y + (long long)p.ny * c.z, L::opp(i)};
  const int sx = wrap_add(c.x, -L::cx(i), p.nx);
  const int sy = wrap_add(c.y, -L::cy(i), p.ny);
  const int sz = wrap_add(c.z, -L::cz(i), p.nz);
  return {sx, (long long)sy + (long long)p.ny * sz, i};
}

// Byte offset of population i of component k at the site itself.
template <class S, int LAT, typename T>
__device__ __forceinline__ uint64_t own_byte(const SiteCoord& c, int k, int i, const Params<T>& p) {
  return pop_byte<S, Lattice<LAT>::Q>(p.n, p.nbx, k, i, c.x, (long long)c.y + (long long)p.ny * c.z);
}

// Populations of component k pulled into site c, decoded to the working
// precision, and their running sum (take_slot, take_shifted).
template <class S, int LAT>
__device__ __forceinline__ void pull_pops(const void* fin, const SiteCoord& c, int k,
                                          const Params<typename S::T>& p,
                                          typename S::T (&f)[Lattice<LAT>::Q], typename S::T& sum) {
  using T = typename S::T;
  constexpr int Q = Lattice<LAT>::Q;
  sum = T(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const SlotAt a = pull_slot<LAT>(c, i, p);
    const uint64_t at = pop_byte<S, Q>(p.n, p.nbx, k, a.i, a.x, a.row);
    if constexpr (S::kShift) {
      const _Float16 h = load_half(fin, ref_byte<S, Q>(p.n, p.nbx, k, a.x, a.row));
      if (i == 0)
        take_shifted<LAT>(0, _Float16(0), load_f32(fin, at), h, p.sh.scale[k], p.sh.one, sum, f[i]);
      else
        take_shifted<LAT>(i, load_half(fin, at), 0.f, h, p.sh.scale[k], p.sh.one, sum, f[i]);
    } else {
      take_slot<S, LAT>(i, load_slot<S>(fin, at, i), sum, f[i]);
    }
  }
}

// Populations of component k pulled into site c, exactly, in FP64.
template <class S, int LAT, typename PT>
__device__ __forceinline__ void pull_pops_exact(const void* fin, const SiteCoord& c, int k, const Params<PT>& p,
                                                double (&f)[Lattice<LAT>::Q]) {
  constexpr int Q = Lattice<LAT>::Q;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const SlotAt a = pull_slot<LAT>(c, i, p);
    const auto raw = load_slot<S>(fin, pop_byte<S, Q>(p.n, p.nbx, k, a.i, a.x, a.row), i);
    float h = 0.f;
    if constexpr (S::kShift) h = float(load_half(fin, ref_byte<S, Q>(p.n, p.nbx, k, a.x, a.row)));
    f[i] = take_exact<S, LAT>(i, raw, h, p.sh.scale[k]);
  }
}

// Store the post-collision populations of component k at site c.  Plain
// codecs write the values; the shifted codec writes the site's new
// reference, the FP16 deviations of the moving populations, and in slot 0
// the rest of the ledger (`sum`: the pulled total in units of s).
template <class S, int LAT>
__device__ __forceinline__ void store_pops(void* fout, const SiteCoord& c, int k, const Params<typename S::T>& p,
                                           const typename S::T (&post)[Lattice<LAT>::Q], typename S::T sum) {
  using T = typename S::T;
  constexpr int Q = Lattice<LAT>::Q;
  char* out = static_cast<char*>(fout);
  if constexpr (S::kShift) {
    const _Float16 h = new_ref(sum);
    _Float16 d[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      d[i] = encode_move<LAT>(i, post[i], p.sh.inv_scale[k], float(h));
      *reinterpret_cast<_Float16*>(out + own_byte<S, LAT>(c, k, i, p)) = d[i];
    }
    *reinterpret_cast<_Float16*>(out + ref_byte<S, Q>(p.n, p.nbx, k, c.x, (long long)c.y + (long long)p.ny * c.z)) = h;
    *reinterpret_cast<float*>(out + own_byte<S, LAT>(c, k, 0, p)) = ledger_rest<Q>(sum, float(h), d, p.sh.minus_one);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) *reinterpret_cast<T*>(out + own_byte<S, LAT>(c, k, i, p)) = post[i];
  }
}

// ---------------------------------------------------------------- init ----
// Rest equilibrium f_i(r, 0) = w_i rho0(r), written in pull storage: slot
// (i, r) holds the value that arrives at r + v_i (at r itself when a wall
// lies between: the value pulled back across the wall).  The shifted codec
// gives each site the reference of T0 = rho0 / s on the 2^-24 grid, stores
// the FP16 deviations of the moving slots against it, and puts in the rest
// slot of r what makes the total pulled into r equal T0(r) exactly (the
// slots pulled into r are re-encoded here exactly as their own sites write
// them).
template <class S, int LAT>
__global__ void __launch_bounds__(kBlock) k_init(const double* __restrict__ rho0, void* __restrict__ f,
                                                 Params<typename S::T> p) {
  using L = Lattice<LAT>;
  using T = typename S::T;
  constexpr int Q = L::Q;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.S) return;
  const SiteCoord c = coord_of(s, p);
  char* out = static_cast<char*>(f);
  for (int k = 0; k < p.n; ++k) {
    const double* rk = rho0 + (long long)k * p.S;
    if constexpr (S::kShift) {
      const double inv_s = double(p.sh.inv_scale[k]);
      // T0 and the reference of a site
      auto total = [&](long long site) { return rint(rk[site] * inv_s * 16777216.0) / 16777216.0; };
      auto ref_of = [&](long long site) { return new_ref(float(total(site))); };
      const _Float16 h = ref_of(s);
      double rest = total(s) - double(ref_weight<LAT>(0)) * double(float(h));
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        // the slot written here carries w_i rho0(r + v_i)
        const double rn = rk[stream_target<LAT>(c, i, p)];
        *reinterpret_cast<_Float16*>(out + own_byte<S, LAT>(c, k, i, p)) =
            encode_move<LAT>(i, float(L::w(i) * rn), p.sh.inv_scale[k], float(h));
        // the slot pulled into r carries w_i rho0(r), against its site's reference
        const SlotAt a = pull_slot<LAT>(c, i, p);
        const long long src = (long long)a.x + (long long)p.nx * a.row;
        const float hs = float(ref_of(src));
        const float d = float(encode_move<LAT>(i, float(L::w(i) * rk[s]), p.sh.inv_scale[k], hs));
        rest -= double(ref_weight<LAT>(i)) * double(hs) + double(d);
      }
      *reinterpret_cast<_Float16*>(out + ref_byte<S, Q>(p.n, p.nbx, k, c.x, (long long)c.y + (long long)p.ny * c.z)) = h;
      *reinterpret_cast<float*>(out + own_byte<S, LAT>(c, k, 0, p)) = float(rest);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const long long src = stream_target<LAT>(c, i, p);
        *reinterpret_cast<T*>(out + own_byte<S, LAT>(c, k, i, p)) = T(L::w(i) * rk[src]);
      }
    }
  }
}

// ------------------------------------------------------------- density ----
// rho^sigma(r) = sum_i f_i(r): the population at r in direction i is the
// slot (i, r - v_i).  The step takes it in the working precision (plain
// codecs: the sum in direction order; shifted codec: s times the exact total); the
// observables take the exact stored values summed in FP64.
// NC > 0: the component count as a template parameter (N = NC), so that
// all components' loads can be issued together (used on D3Q19, where it
// makes the shifted FP16 density pass 20% faster; on D2Q9 the runtime loop
// is faster); 0: any N.
template <class S, int LAT, typename TO, int NC = 0>
__global__ void __launch_bounds__(kBlock) k_density(const void* __restrict__ f, TO* __restrict__ rho,
                                                    Params<typename S::T> p) {
  using L = Lattice<LAT>;
  using T = typename S::T;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.S) return;
  const SiteCoord c = coord_of(s, p);
  const int n = NC > 0 ? NC : p.n;
#pragma unroll
  for (int k = 0; k < (NC > 0 ? NC : kMaxComp); ++k) {
    if (k >= n) break;
    if constexpr (sizeof(TO) > sizeof(T)) {
      double v[L::Q];
      pull_pops_exact<S, LAT>(f, c, k, p, v);
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < L::Q; ++i) acc += v[i];
      rho[(long long)k * p.S + s] = acc;
    } else {
      T v[L::Q], sum;
      pull_pops<S, LAT>(f, c, k, p, v, sum);
      rho[(long long)k * p.S + s] = site_density<S>(sum, p.sh.scale[k]);
    }
  }
}

// ----------------------------------------------------------- potential ----
// lap rho^sigma = 6 sum_i w_i (rho^sigma(r + v_i) - rho^sigma(r)), then the
// chemical potentials and the potential h^sigma the force differentiates.
// NC: compile-time bound on the component count (kMaxComp for any N, or N
// itself); entries from p.n up are padding that the potential ignores.
template <int LAT, typename T, int NC = kMaxComp>
__global__ void __launch_bounds__(kBlock) k_potential(const T* __restrict__ rho, T* __restrict__ mu_out,
                                                      T* __restrict__ h_out, Params<T> p) {
  using L = Lattice<LAT>;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.S) return;
  const SiteCoord c = coord_of(s, p);
  long long nb[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) nb[i] = neighbour<LAT>(c, i, +1, p);
  T r[NC], lap[NC], mu[NC], h[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    r[k] = T(1);
    lap[k] = T(0);
    if (k < p.n) {
      const T* rk = rho + (long long)k * p.S;
      r[k] = rk[s];
      lap[k] = lattice_laplacian<LAT, T>([&](int i) { return rk[nb[i]]; }, r[k]);
    }
  }
  // NC < kMaxComp: instantiated for N itself (the run-time guards on N go)
  site_potential<T, NC, (NC < kMaxComp)>(p, r, lap, mu, h);
  for (int k = 0; k < p.n; ++k) {
    if (mu_out) mu_out[(long long)k * p.S + s] = mu[k];
    h_out[(long long)k * p.S + s] = h[k];
  }
}

// ------------------------------------------------------------- collide ----
template <class S, int LAT>
__global__ void __launch_bounds__(kBlock) k_collide(const void* __restrict__ fin, void* __restrict__ fout,
                                                    const typename S::T* __restrict__ rho,
                                                    const typename S::T* __restrict__ h, Params<typename S::T> p) {
  using L = Lattice<LAT>;
  using T = typename S::T;
  constexpr int Q = L::Q;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.S) return;
  const SiteCoord c = coord_of(s, p);
  long long nb[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) nb[i] = neighbour<LAT>(c, i, +1, p);
  // barycentric velocity u = sum_sigma j^sigma / sum_sigma rho^sigma
  T jx[kMaxComp], jy[kMaxComp], jz[kMaxComp];
  T rt = T(0), ux = T(0), uy = T(0), uz = T(0);
  for (int k = 0; k < p.n; ++k) {
    T f[Q], sum;
    pull_pops<S, LAT>(fin, c, k, p, f, sum);
    T ax = T(0), ay = T(0), az = T(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (L::cx(i)) ax += T(L::cx(i)) * f[i];
      if (L::cy(i)) ay += T(L::cy(i)) * f[i];
      if (L::cz(i)) az += T(L::cz(i)) * f[i];
    }
    jx[k] = ax;
    jy[k] = ay;
    jz[k] = az;
    ux += ax;
    uy += ay;
    uz += az;
    rt += rho[(long long)k * p.S + s];
  }
  const T inv_rt = rcp_(rt);
  ux *= inv_rt;
  uy *= inv_rt;
  uz *= inv_rt;
  for (int k = 0; k < p.n; ++k) {
    const T rs = rho[(long long)k * p.S + s];
    T f[Q], sum;
    pull_pops<S, LAT>(fin, c, k, p, f, sum);
    const T* hk = h + (long long)k * p.S;
    const T* rk = rho + (long long)k * p.S;
    T Ax, Ay, Az;
    lattice_force<LAT, T>([&](int i) { return hk[nb[i]]; }, [&](int i) { return rk[nb[i]]; }, rs, p, Ax, Ay,
                          Az);
    const T inv_rs = rcp_(rs);
    collide<LAT, T>(f, rs, ux, uy, uz, Ax, Ay, Az, jx[k] * inv_rs, jy[k] * inv_rs, jz[k] * inv_rs,
                    p.inv_tau);
    store_pops<S, LAT>(fout, c, k, p, f, sum);
  }
}

// The same step for a compile-time component count (N <= 4): each
// component's pulled populations are loaded once and stay in registers from
// the barycentric velocity to the collision (k_collide loads them twice,
// which on large 3D lattices means twice from HBM).  Same operations in the
// same order, so the same bits.
template <class S, int LAT, int NC>
__global__ void __launch_bounds__(kBlock) k_collide_nc(const void* __restrict__ fin, void* __restrict__ fout,
                                                       const typename S::T* __restrict__ rho,
                                                       const typename S::T* __restrict__ h,
                                                       Params<typename S::T> p) {
  using L = Lattice<LAT>;
  using T = typename S::T;
  constexpr int Q = L::Q;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.S) return;
  const SiteCoord c = coord_of(s, p);
  long long nb[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) nb[i] = neighbour<LAT>(c, i, +1, p);
  T f[NC][Q], led[NC];
  T jx[NC], jy[NC], jz[NC];
  T rt = T(0), ux = T(0), uy = T(0), uz = T(0);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    pull_pops<S, LAT>(fin, c, k, p, f[k], led[k]);
    T ax = T(0), ay = T(0), az = T(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (L::cx(i)) ax += T(L::cx(i)) * f[k][i];
      if (L::cy(i)) ay += T(L::cy(i)) * f[k][i];
      if (L::cz(i)) az += T(L::cz(i)) * f[k][i];
    }
    jx[k] = ax;
    jy[k] = ay;
    jz[k] = az;
    ux += ax;
    uy += ay;
    uz += az;
    rt += rho[(long long)k * p.S + s];
  }
  const T inv_rt = rcp_(rt);
  ux *= inv_rt;
  uy *= inv_rt;
  uz *= inv_rt;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const T rs = rho[(long long)k * p.S + s];
    const T* hk = h + (long long)k * p.S;
    const T* rk = rho + (long long)k * p.S;
    T Ax, Ay, Az;
    lattice_force<LAT, T>([&](int i) { return hk[nb[i]]; }, [&](int i) { return rk[nb[i]]; }, rs, p, Ax, Ay,
                          Az);
    const T inv_rs = rcp_(rs);
    collide<LAT, T>(f[k], rs, ux, uy, uz, Ax, Ay, Az, jx[k] * inv_rs, jy[k] * inv_rs, jz[k] * inv_rs,
                    p.inv_tau);
    store_pops<S, LAT>(fout, c, k, p, f[k], led[k]);
  }
}

// --------------------------------------------------------- observables ----
// U = u + (1/2) sum A / rho, and the pressure tensor
//   P_ab = [p0 - kappa sum_s (rho lap rho + |grad rho|^2 / 2)] d_ab
//        + kappa sum_s d_a rho d_b rho,     p0 = sum_s rho mu0 - psi,
// all in FP64 from the stored populations (converted exactly to FP64).
template <class S, int LAT>
__global__ void __launch_bounds__(kBlock) k_observe(const void* __restrict__ fin, const double* __restrict__ rho,
                                                    const double* __restrict__ h, double* __restrict__ U,
                                                    double* __restrict__ P, Params<double> p) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.S) return;
  const SiteCoord c = coord_of(s, p);
  long long nb[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) nb[i] = neighbour<LAT>(c, i, +1, p);
  double rt = 0, jt[3] = {0, 0, 0}, At[3] = {0, 0, 0};
  double r[kMaxComp], lap[kMaxComp], g[kMaxComp][3];
  for (int k = 0; k < kMaxComp; ++k) {
    r[k] = 1.0;
    lap[k] = 0.0;
    g[k][0] = g[k][1] = g[k][2] = 0.0;
  }
  for (int k = 0; k < p.n; ++k) {
    double fk[Q];
    pull_pops_exact<S, LAT>(fin, c, k, p, fk);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      jt[0] += L::cx(i) * fk[i];
      jt[1] += L::cy(i) * fk[i];
      jt[2] += L::cz(i) * fk[i];
    }
    const double* rk = rho + (long long)k * p.S;
    r[k] = rk[s];
    rt += r[k];
    const double* hk = h + (long long)k * p.S;
    double Ax, Ay, Az;
    lattice_force<LAT, double>([&](int i) { return hk[nb[i]]; }, [&](int i) { return rk[nb[i]]; }, r[k], p,
                               Ax, Ay, Az);
    At[0] += Ax;
    At[1] += Ay;
    At[2] += Az;
    double acc = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const double rv = rk[nb[i]];
      acc += L::w(i) * (rv - r[k]);
      g[k][0] += 3.0 * L::w(i) * L::cx(i) * rv;
      g[k][1] += 3.0 * L::w(i) * L::cy(i) * rv;
      g[k][2] += 3.0 * L::w(i) * L::cz(i) * rv;
    }
    lap[k] = 6.0 * acc;
  }
  for (int a = 0; a < D; ++a) U[(long long)a * p.S + s] = (jt[a] + 0.5 * At[a]) / rt;
  // bulk pressure from the potential without the gradient term
  Params<double> pb = p;
  pb.kappa = 0.0;
  double zero[kMaxComp], mu0[kMaxComp], h0[kMaxComp];
  for (int k = 0; k < kMaxComp; ++k) zero[k] = 0.0;
  site_potential<double, kMaxComp>(pb, r, zero, mu0, h0);
  double p0 = -site_psi<double, kMaxComp>(pb, r), iso = 0.0;
  for (int k = 0; k < p.n; ++k) {
    p0 += r[k] * mu0[k];
    iso += r[k] * lap[k] + 0.5 * (g[k][0] * g[k][0] + g[k][1] * g[k][1] + g[k][2] * g[k][2]);
  }
  int m = 0;
  for (int a = 0; a < D; ++a)
    for (int b = a; b < D; ++b) {
      double gg = 0;
      for (int k = 0; k < p.n; ++k) gg += g[k][a] * g[k][b];
      double v = p.kappa * gg;
      if (a == b) v += p0 - p.kappa * iso;
      P[(long long)m * p.S + s] = v;
      ++m;
    }
}

// Populations at the current time, FP64 [N][Q][S].
template <class S, int LAT>
__global__ void __launch_bounds__(kBlock) k_unpull(const void* __restrict__ fin, double* __restrict__ out,
                                                   Params<typename S::T> p) {
  using L = Lattice<LAT>;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.S) return;
  const SiteCoord c = coord_of(s, p);
  for (int k = 0; k < p.n; ++k) {
    double fk[L::Q];
    pull_pops_exact<S, LAT>(fin, c, k, p, fk);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) out[((long long)k * L::Q + i) * p.S + s] = fk[i];
  }
}

// ---------------------------------------------------------- diagnostics ----
// Per block: FP64 sums of rho^sigma (N values), of the first moments over
// components (D values), and a flag (1 if any rho^sigma is NaN or <= 0).
// Wave64 butterfly reduction, then the waves of the block in index order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <class S, int LAT>
__global__ void __launch_bounds__(kBlock) k_diag(const void* __restrict__ fin, double* __restrict__ partial,
                                                 Params<typename S::T> p) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D;
  constexpr int K = kMaxComp + D + 1;
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < p.S;
       s += (long long)gridDim.x * blockDim.x) {
    const SiteCoord c = coord_of(s, p);
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) {
      if (k < p.n) {
        double fk[Q];
        pull_pops_exact<S, LAT>(fin, c, k, p, fk);
        double r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const double fi = fk[i];
          r += fi;
          jx += L::cx(i) * fi;
          jy += L::cy(i) * fi;
          jz += L::cz(i) * fi;
        }
        acc[k] += r;
        acc[kMaxComp] += jx;
        if constexpr (D > 1) acc[kMaxComp + 1] += jy;
        if constexpr (D > 2) acc[kMaxComp + 2] += jz;
        if (!(r > 0.0) || !(r < 1e300)) acc[K - 1] = 1.0;
      }
    }
  }
  __shared__ double red[kBlock / 64][K];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < K - 1; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[wave][q] = v;
  }
  // the flag is a maximum, not a sum
  double fl = acc[K - 1];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) fl = fmax(fl, __shfl_xor(fl, off, 64));
  if (lane == 0) red[wave][K - 1] = fl;
  __syncthreads();
  if (threadIdx.x < K) {
    double v = 0.0;
    for (int wv = 0; wv < kBlock / 64; ++wv)
      v = (threadIdx.x == K - 1) ? fmax(v, red[wv][threadIdx.x]) : v + red[wv][threadIdx.x];
    partial[(long long)blockIdx.x * K + threadIdx.x] = v;
  }
}

// Sum the block partials in block order (one thread per quantity), store
// the totals, and OR the flag into the sticky health flag.
__global__ void k_diag_final(const double* __restrict__ partial, int nblocks, int K,
                             double* __restrict__ out, int* __restrict__ flag) {
  const int q = threadIdx.x;
  if (q >= K) return;
  double v = 0.0;
  for (int b = 0; b < nblocks; ++b) {
    const double x = partial[(long long)b * K + q];
    v = (q == K - 1) ? fmax(v, x) : v + x;
  }
  out[q] = v;
  if (q == K - 1 && v != 0.0) flag[0] = 1;
}

// ------------------------------------------------------------ launchers ----
static inline unsigned grid_for(long long S) { return unsigned((S + kBlock - 1) / kBlock); }

template <class S, int LAT>
struct SplitOps {
  using T = typename S::T;
  static void init(const Ctx& c, const double* rho0_dev, void* f) {
    k_init<S, LAT><<<grid_for(c.S), kBlock, 0, c.stream>>>(rho0_dev, f, c.params<T>());
  }
  static void step(const Ctx& c, const void* fin, void* fout) {
    const Params<T>& p = c.params<T>();
    T* rho = static_cast<T*>(c.rho_scratch);
    T* h = static_cast<T*>(c.h_scratch);
    const unsigned g = grid_for(c.S);
    bool density_done = false;
    if constexpr (LAT == 3) {
      density_done = true;
      switch (p.n) {
        case 1: k_density<S, LAT, T, 1><<<g, kBlock, 0, c.stream>>>(fin, rho, p); break;
        case 2: k_density<S, LAT, T, 2><<<g, kBlock, 0, c.stream>>>(fin, rho, p); break;
        case 3: k_density<S, LAT, T, 3><<<g, kBlock, 0, c.stream>>>(fin, rho, p); break;
        case 4: k_density<S, LAT, T, 4><<<g, kBlock, 0, c.stream>>>(fin, rho, p); break;
        default: density_done = false;
      }
    }
    if (!density_done) k_density<S, LAT, T><<<g, kBlock, 0, c.stream>>>(fin, rho, p);
    switch (p.n) {
      case 1:
        k_potential<LAT, T, 1><<<g, kBlock, 0, c.stream>>>(rho, nullptr, h, p);
        k_collide_nc<S, LAT, 1><<<g, kBlock, 0, c.stream>>>(fin, fout, rho, h, p);
        break;
      case 2:
        k_potential<LAT, T, 2><<<g, kBlock, 0, c.stream>>>(rho, nullptr, h, p);
        k_collide_nc<S, LAT, 2><<<g, kBlock, 0, c.stream>>>(fin, fout, rho, h, p);
        break;
      case 3:
        k_potential<LAT, T, 3><<<g, kBlock, 0, c.stream>>>(rho, nullptr, h, p);
        k_collide_nc<S, LAT, 3><<<g, kBlock, 0, c.stream>>>(fin, fout, rho, h, p);
        break;
      case 4:
        k_potential<LAT, T, 4><<<g, kBlock, 0, c.stream>>>(rho, nullptr, h, p);
        k_collide_nc<S, LAT, 4><<<g, kBlock, 0, c.stream>>>(fin, fout, rho, h, p);
        break;
      default:
        k_potential<LAT, T><<<g, kBlock, 0, c.stream>>>(rho, nullptr, h, p);
        k_collide<S, LAT><<<g, kBlock, 0, c.stream>>>(fin, fout, rho, h, p);
    }
  }
  static void observe(const Ctx& c, const void* fin, double* rho, double* mu, double* h, double* U,
                      double* P) {
    k_density<S, LAT, double><<<grid_for(c.S), kBlock, 0, c.stream>>>(fin, rho, c.params<T>());
    k_potential<LAT, double><<<grid_for(c.S), kBlock, 0, c.stream>>>(rho, mu, h, c.pd);
    k_observe<S, LAT><<<grid_for(c.S), kBlock, 0, c.stream>>>(fin, rho, h, U, P, c.pd);
  }
  static void unpull(const Ctx& c, const void* fin, double* out) {
    k_unpull<S, LAT><<<grid_for(c.S), kBlock, 0, c.stream>>>(fin, out, c.params<T>());
  }
  static void diag(const Ctx& c, const void* fin) {
    constexpr int K = kMaxComp + Lattice<LAT>::D + 1;
    k_diag<S, LAT><<<c.diag_blocks, kBlock, 0, c.stream>>>(fin, c.diag_partial, c.params<T>());
    k_diag_final<<<1, 64, 0, c.stream>>>(c.diag_partial, c.diag_blocks, K, c.diag_out, c.health_flag);
  }
};

template <class S>
static const SplitTable& table_for_lattice(int lattice) {
  static const SplitTable t1 = {SplitOps<S, 1>::init, SplitOps<S, 1>::step, SplitOps<S, 1>::observe,
                                SplitOps<S, 1>::unpull, SplitOps<S, 1>::diag};
  static const SplitTable t2 = {SplitOps<S, 2>::init, SplitOps<S, 2>::step, SplitOps<S, 2>::observe,
                                SplitOps<S, 2>::unpull, SplitOps<S, 2>::diag};
  static const SplitTable t3 = {SplitOps<S, 3>::init, SplitOps<S, 3>::step, SplitOps<S, 3>::observe,
                                SplitOps<S, 3>::unpull, SplitOps<S, 3>::diag};
  return lattice == 1 ? t1 : (lattice == 2 ? t2 : t3);
}

const SplitTable& split_table(int lattice, int storage) {
  switch (storage) {
    case StoreF64::kId: return table_for_lattice<StoreF64>(lattice);
    case StoreF32::kId: return table_for_lattice<StoreF32>(lattice);
    default: return table_for_lattice<StoreF16S>(lattice);
  }
}

}  // namespace lbm
