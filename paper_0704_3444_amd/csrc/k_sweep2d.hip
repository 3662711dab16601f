// Strip-sweep D2Q9 step: one launch per time step, every population read
// once and written once, with almost no halo re-reads.
//
// A workgroup of four waves owns a strip of 64 columns (one 64-site block of
// the population layout) and a segment of rows, which it sweeps from top to
// bottom.  Wave w handles the rows y = w (mod 4) of the segment.  One round
// advances four rows:
//   1. density rho^sigma of the rows one round ahead, from populations the
//      waves already hold in registers (plus four halo columns formed by 12
//      lanes), into an LDS ring of rows;
//   2. chemical potentials and the potential h of four rows into an LDS ring
//      (the Laplacian in mu and the gradient of mu reach two rows ahead);
//   3. prefetch of the populations two rounds ahead;
//   4. force, equilibrium, forcing term and collision of the current row,
//      stored in place (streaming happens through the next step's pull).
// Each wave keeps three rows of populations in registers (current, one round
// ahead, in flight).  Rows are re-read only at the two ends of a segment
// (4 rows per segment) and the strip edges (4 columns per 64), instead of a
// two-site ring around every tile.  Workgroups are banded per XCD so that
// neighbouring strips share L2.
//
// The kernel is templated on the storage codec (storage.hpp): FP32, or
// shifted FP16 whose rows stay in registers as stored (per component the
// FP32 ledger and four packed pairs of FP16 deviations, 5 registers instead
// of 9) and are decoded where the collision needs them.
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"
#include "physics.hpp"
#include "storage.hpp"

namespace lbm {
namespace sweep {

constexpr int kXcds = 8;
constexpr int kRhoRing = 16;  // rows of rho kept in LDS (live span is 9)
constexpr int kHRing = 8;     // rows of h kept in LDS (live span is 8)
constexpr int kW = 64;        // strip width = block width = wave size
constexpr int kRW = kW + 4;   // rho row: columns x0 - 2 .. x0 + 65
constexpr int kHW = kW + 2;   // h row:   columns x0 - 1 .. x0 + 64

__device__ __forceinline__ int wrap_mod(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Byte offset of the 64-site block that holds site (x, y); the caller
// guarantees one copy is below 4 GiB.
template <class S, int NC>
__device__ __forceinline__ uint32_t blk_off(int nbx, int x, int y) {
  return (uint32_t(y) * uint32_t(nbx) + uint32_t(x >> 6)) * uint32_t(NC * BlockLayout<S, 9>::kComp);
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// Populations of one site for J components as stored.
template <class S, int J>
struct Pops;

template <int J>
struct Pops<StoreF32, J> {
  float v[J][9];
  __device__ __forceinline__ void set(int j, int i, const char* a) { v[j][i] = *reinterpret_cast<const float*>(a); }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < 9; ++i) v[j][i] = 0.0f;
  }
  // density of entry j (component c), summed in direction order
  __device__ __forceinline__ float density(const ShiftRef&, int j, int) const {
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) acc += v[j][i];
    return acc;
  }
  __device__ __forceinline__ void decode(const ShiftRef&, int j, float (&f)[9], float& ledger) const {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = v[j][i];
    ledger = 0.0f;
  }
};

template <int J>
struct Pops<StoreF16S, J> {
  float r[J];          // ledger slot (i = 0)
  half2_t m[J][4];     // deviations of i = 1 .. 8, two per register
  __device__ __forceinline__ void set(int j, int i, const char* a) {
    if (i == 0)
      r[j] = *reinterpret_cast<const float*>(a);
    else
      m[j][(i - 1) >> 1][(i - 1) & 1] = *reinterpret_cast<const _Float16*>(a);
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      r[j] = 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) m[j][k] = half2_t{_Float16(0), _Float16(0)};
    }
  }
  __device__ __forceinline__ float raw(int j, int i) const {
    return i == 0 ? r[j] : float(m[j][(i - 1) >> 1][(i - 1) & 1]);
  }
  // exact total deviation d_0 + sum_{i>0} d_i, in direction order
  __device__ __forceinline__ float ledger(int j) const {
    float L = r[j];
#pragma unroll
    for (int i = 1; i < 9; ++i) L += raw(j, i);
    return L;
  }
  __device__ __forceinline__ float density(const ShiftRef& sh, int j, int c) const {
    return __builtin_fmaf(ledger(j), sh.scale[c], sh.csum[c]);
  }
  __device__ __forceinline__ void decode(const ShiftRef& sh, int j, float (&f)[9], float& L) const {
    L = ledger(j);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = ::lbm::decode<StoreF16S, 2>(sh, j, i, raw(j, i));
  }
};

// The populations pulled into site (x, prow): f_i comes from (x - v_i).
template <class S, int NC>
__device__ __forceinline__ void load_row(const void* __restrict__ fin, const Params<float>& p, int x, int prow,
                                         Pops<S, NC>& F) {
  using L = Lattice<2>;
  using B = BlockLayout<S, 9>;
  const char* base = static_cast<const char*>(fin);
  const int xm = wrap_add(x, -1, p.nx), xp = wrap_add(x, 1, p.nx);
  const int ym = wrap_add(prow, -1, p.ny), yp = wrap_add(prow, 1, p.ny);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int sx = L::cx(i) > 0 ? xm : (L::cx(i) < 0 ? xp : x);
    const int sy = L::cy(i) > 0 ? ym : (L::cy(i) < 0 ? yp : prow);
    const uint32_t off = blk_off<S, NC>(p.nbx, sx, sy) + B::in_run(i, sx);
#pragma unroll
    for (int c = 0; c < NC; ++c) F.set(c, i, base + off + B::run(c, i));
  }
}

// Halo columns x0-2, x0-1, x0+64, x0+65 of the four rows r0 .. r0+3: lane
// L < 16 NC pulls the nine populations of (row r0 + L / (4 NC), halo column,
// component).  One wave loads them for the whole workgroup.
template <class S, int NC>
__device__ __forceinline__ void load_halo4(const void* __restrict__ fin, const Params<float>& p, int lane, int x0,
                                           int r0, Pops<S, 1>& Hv) {
  using L = Lattice<2>;
  using B = BlockLayout<S, 9>;
  const char* base = static_cast<const char*>(fin);
  if (lane < 16 * NC) {
    const int wr = lane / (4 * NC), hc = (lane % (4 * NC)) / NC, c = lane % NC;
    const int prow = wrap_mod(r0 + wr, p.ny);
    const int hx = wrap_mod(x0 + (hc < 2 ? hc - 2 : kW + hc - 2), p.nx);
    const int xm = wrap_add(hx, -1, p.nx), xp = wrap_add(hx, 1, p.nx);
    const int ym = wrap_add(prow, -1, p.ny), yp = wrap_add(prow, 1, p.ny);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int sx = L::cx(i) > 0 ? xm : (L::cx(i) < 0 ? xp : hx);
      const int sy = L::cy(i) > 0 ? ym : (L::cy(i) < 0 ? yp : prow);
      Hv.set(0, i, base + blk_off<S, NC>(p.nbx, sx, sy) + B::in_run(i, sx) + B::run(c, i));
    }
  }
}

template <class S, int NC, int PF>
__global__ void __launch_bounds__(256) k_sweep_d2q9(const void* __restrict__ fin, void* __restrict__ fout,
                                                    Params<float> p, int strips, int seg_rows, int ntiles,
                                                    int tiles_per_xcd) {
  using L = Lattice<2>;
  using T = float;
  using B = BlockLayout<S, 9>;
  static_assert(PF == 1 || PF == 2, "prefetch depth in rounds");
  __shared__ T s_rho[kRhoRing][NC][kRW];
  __shared__ T s_h[kHRing][NC][kHW];

  const int b = blockIdx.x;
  const int t = (b % kXcds) * tiles_per_xcd + b / kXcds;
  if (t >= ntiles) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int x0 = (t % strips) * kW;
  const int ya = (t / strips) * seg_rows;
  const int yb = min(ya + seg_rows, p.ny);
  const int rounds = (yb - ya + 3) / 4;
  const int x = x0 + lane;  // nx is a multiple of 64: every lane is a site
  const int ny = p.ny;
  constexpr int kHaloWave = 1, kEdgeWave = 0;

  // ring slots of virtual row r (r >= ya - 8 always)
  auto rslot = [&](int r) { return (r - ya + 8 * kRhoRing) & (kRhoRing - 1); };
  auto hslot = [&](int r) { return (r - ya + 8 * kHRing) & (kHRing - 1); };

  // density of virtual row r from the wave's populations
  auto put_rho = [&](int r, const Pops<S, NC>& F) {
    const int sr = rslot(r);
#pragma unroll
    for (int c = 0; c < NC; ++c) s_rho[sr][c][lane + 2] = F.density(p.sh, c, c);
  };
  // halo densities of rows r0 .. r0+3 from the halo wave's values
  auto put_rho_halo = [&](int r0, const Pops<S, 1>& Hv) {
    if (lane < 16 * NC) {
      const int wr = lane / (4 * NC), hc = (lane % (4 * NC)) / NC, c = lane % NC;
      s_rho[rslot(r0 + wr)][c][hc < 2 ? hc : kW + hc] = Hv.density(p.sh, 0, c);
    }
  };

  // potential h of virtual row r at h position q (column x0 - 1 + q)
  auto put_h = [&](int r, int q) {
    const int s0 = rslot(r - 1), s1 = rslot(r), s2 = rslot(r + 1);
    const int pc = q + 1;  // rho position of the column
    T rr[NC], lap[NC], mu[NC], hh[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      rr[c] = s_rho[s1][c][pc];
      lap[c] = lattice_laplacian<2, T>(
          [&](int i) {
            const int sy = L::cy(i) > 0 ? s2 : (L::cy(i) < 0 ? s0 : s1);
            return s_rho[sy][c][pc + L::cx(i)];
          },
          rr[c]);
    }
    site_potential<T, NC>(p, rr, lap, mu, hh);
    const int sh = hslot(r);
#pragma unroll
    for (int c = 0; c < NC; ++c) s_h[sh][c][q] = hh[c];
  };
  // h of rows r0 .. r0+3: each wave its own row's 64 interior columns, the
  // edge wave the eight edge columns (q = 0 and 65) of all four rows
  auto put_h4 = [&](int r0) {
    put_h(r0 + w, lane + 1);
    if (w == kEdgeWave && lane < 8) put_h(r0 + (lane >> 1), (lane & 1) ? kHW - 1 : 0);
  };

  // F[0]: row collided this round; F[1 .. PF]: rows whose density is formed
  // in the next rounds (in flight); F[PF + 1]: the row prefetched this round.
  // Hv[0 .. PF - 1]: halo values of the rows of F[1 .. PF]; Hv[PF] prefetched.
  Pops<S, NC> F[PF + 2];
  Pops<S, 1> Hv[PF + 1];
#pragma unroll
  for (int s = 0; s <= PF; ++s) Hv[s].zero();

  // ---- prologue --------------------------------------------------------
  // rho of rows ya-2, ya-1 (waves 2, 3) and ya .. ya+3 (all waves); h of rows
  // ya-1 .. ya+2; populations of row ya + w (collided in round 0) in F[0] and
  // of rows ya + 4j + w, j = 1 .. PF, in flight.
  if (w >= 2) load_row<S, NC>(fin, p, x, wrap_mod(ya - 4 + w, ny), F[1]);
  if (w == kHaloWave) load_halo4<S, NC>(fin, p, lane, x0, ya - 4, Hv[0]);
  if (w >= 2) put_rho(ya - 4 + w, F[1]);
  if (w == kHaloWave) put_rho_halo(ya - 4, Hv[0]);
  load_row<S, NC>(fin, p, x, wrap_mod(ya + w, ny), F[0]);
  if (w == kHaloWave) load_halo4<S, NC>(fin, p, lane, x0, ya, Hv[0]);
  put_rho(ya + w, F[0]);
  if (w == kHaloWave) put_rho_halo(ya, Hv[0]);
  __syncthreads();
  put_h4(ya - 1);
  __syncthreads();
#pragma unroll
  for (int j = 1; j <= PF; ++j) {
    load_row<S, NC>(fin, p, x, wrap_mod(ya + 4 * j + w, ny), F[j]);
    if (w == kHaloWave) load_halo4<S, NC>(fin, p, lane, x0, ya + 4 * j, Hv[j - 1]);
  }

  // ---- rounds ------------------------------------------------------------
  for (int k = 0; k < rounds; ++k) {
    const int rc = ya + 4 * k + w;  // row collided by this wave
    const int ra = rc + 4;          // row whose density is formed this round
    put_rho(ra, F[1]);
    if (w == kHaloWave) put_rho_halo(ya + 4 * k + 4, Hv[0]);
    __syncthreads();
    put_h4(ya + 4 * k + 3);
    __syncthreads();
    if (k + PF < rounds) {
      load_row<S, NC>(fin, p, x, wrap_mod(ra + 4 * PF, ny), F[PF + 1]);
      if (w == kHaloWave) load_halo4<S, NC>(fin, p, lane, x0, ya + 4 * k + 4 + 4 * PF, Hv[PF]);
    }
    if (rc < yb) {
      const int sr = rslot(rc);
      T rs[NC], jx[NC], jy[NC];
      T rt = T(0), ux = T(0), uy = T(0);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T f[9], ledger;
        F[0].decode(p.sh, c, f, ledger);
        T ax = T(0), ay = T(0);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          if (L::cx(i)) ax += T(L::cx(i)) * f[i];
          if (L::cy(i)) ay += T(L::cy(i)) * f[i];
        }
        jx[c] = ax;
        jy[c] = ay;
        rs[c] = s_rho[sr][c][lane + 2];
        ux += ax;
        uy += ay;
        rt += rs[c];
      }
      const T inv_rt = rcp_(rt);
      ux *= inv_rt;
      uy *= inv_rt;
      const int h0 = hslot(rc - 1), h1 = hslot(rc), h2 = hslot(rc + 1);
      const int r0 = rslot(rc - 1), r2 = rslot(rc + 1);
      char* own = static_cast<char*>(fout) + blk_off<S, NC>(p.nbx, x, rc);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T Ax, Ay, Az;
        lattice_force<2, T>(
            [&](int i) {
              const int sy = L::cy(i) > 0 ? h2 : (L::cy(i) < 0 ? h0 : h1);
              return s_h[sy][c][lane + 1 + L::cx(i)];
            },
            [&](int i) {
              const int sy = L::cy(i) > 0 ? r2 : (L::cy(i) < 0 ? r0 : sr);
              return s_rho[sy][c][lane + 2 + L::cx(i)];
            },
            rs[c], p, Ax, Ay, Az);
        const T inv_rs = rcp_(rs[c]);
        T f[9], ledger;
        F[0].decode(p.sh, c, f, ledger);
        collide<2, T>(f, rs[c], ux, uy, T(0), Ax, Ay, Az, jx[c] * inv_rs, jy[c] * inv_rs, T(0), p.inv_tau);
        if constexpr (S::kShift) {
          // FP16 deviations of the moving populations; the ledger keeps the rest
          T rest = ledger;
#pragma unroll
          for (int i = 1; i < 9; ++i) {
            const _Float16 d = encode_move<2>(p.sh, c, i, f[i]);
            rest -= float(d);
            __builtin_nontemporal_store(d, reinterpret_cast<_Float16*>(own + B::run(c, i) + B::in_run(i, x)));
          }
          __builtin_nontemporal_store(rest, reinterpret_cast<float*>(own + B::run(c, 0) + B::in_run(0, x)));
        } else {
#pragma unroll
          for (int i = 0; i < 9; ++i)
            __builtin_nontemporal_store(f[i], reinterpret_cast<T*>(own + B::run(c, i) + B::in_run(i, x)));
        }
      }
    }
    // rotate the register sets (moves; the rotation is not renamed by unrolling
    // because that needs more registers than one occupancy step allows)
#pragma unroll
    for (int s = 0; s <= PF; ++s) F[s] = F[s + 1];
#pragma unroll
    for (int s = 0; s < PF; ++s) Hv[s] = Hv[s + 1];
  }
}

}  // namespace sweep

// Rows per segment: about one workgroup per resident slot (three per CU on
// 256 CUs), rounded up to whole rounds of four rows, so the grid runs in one
// wave of workgroups and the four rows re-read per segment stay a small
// fraction of it.
static int sweep_rows(int nx, int ny) {
  const int strips = nx / 64;
  const int slots = 3 * 256;
  const int segs = (slots + strips - 1) / strips;
  int rows = (ny + segs - 1) / segs;
  rows = (rows + 3) / 4 * 4;
  return rows < 4 ? 4 : rows;
}

template <class S, int NC>
static void launch_sweep(const Ctx& c, const void* fin, void* fout) {
  const Params<float>& p = c.params<float>();
  const int strips = p.nx / 64;
  const int rows = sweep_rows(p.nx, p.ny);
  const int ntiles = strips * ((p.ny + rows - 1) / rows);
  const int per_xcd = (ntiles + sweep::kXcds - 1) / sweep::kXcds;
  sweep::k_sweep_d2q9<S, NC, 1><<<per_xcd * sweep::kXcds, 256, 0, c.stream>>>(fin, fout, p, strips, rows, ntiles,
                                                                              per_xcd);
}

template <class S>
static FusedStepFn sweep_for_n(int n_comp) {
  switch (n_comp) {
    case 1: return launch_sweep<S, 1>;
    case 2: return launch_sweep<S, 2>;
    case 3: return launch_sweep<S, 3>;
    case 4: return launch_sweep<S, 4>;
    default: return nullptr;
  }
}

// FP32 and shifted FP16 only: three rows of FP64 populations exceed the
// register budget.
FusedStepFn sweep_step_for(int storage, int n_comp) {
  if (storage == StoreF32::kId) return sweep_for_n<StoreF32>(n_comp);
  if (storage == StoreF16S::kId) return sweep_for_n<StoreF16S>(n_comp);
  return nullptr;
}

}  // namespace lbm
