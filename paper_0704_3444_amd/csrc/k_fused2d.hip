// Fused single-kernel D2Q9 step.
//
// One launch per time step.  Each workgroup owns a TX x TY tile of sites and
// runs the whole step of the method for it:
//   A. pull the tile's populations (f_i(r) is slot (i, r - v_i)) into
//      registers and form rho^sigma; stage rho in LDS;
//   B. form rho^sigma on a two-site ring around the tile (the Laplacian in
//      mu and the gradient of mu reach two sites) from the same pulled
//      populations, into LDS; neighbouring workgroups read these rows too,
//      so they come from L2 or the MALL rather than HBM;
//   C. chemical potentials and the potential h on the tile plus one ring,
//      in LDS;
//   D. force, equilibrium, forcing term, BGK collision, and one coalesced
//      store per population at the site itself (streaming happens through
//      the pull of the next step).
// Populations are read once and written once per step from HBM; the stores
// are non-temporal (the next step reads them, long after they would have
// left the caches, and keeping them out preserves L2 for the halo rows).  Workgroup
// indices are remapped so that the eight XCDs (dispatched round-robin) each
// sweep a contiguous band of tiles, keeping halo rows in their own L2.
// No MFMA: the step is a bandwidth-bound stencil, not a contraction.
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"
#include "physics.hpp"
#include "storage.hpp"

namespace lbm {

constexpr int kXcds = 8;

__device__ __forceinline__ int wrap_mod(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// 32-bit byte offset of population 0 of site (x, y); population q sits 64 q
// elements further (the block layout of pop_index).  The host only takes
// this path when one population copy is smaller than 4 GiB, so that every
// access is a uniform 64-bit base plus a 32-bit per-lane offset.
template <typename T>
__device__ __forceinline__ uint32_t site_offset(int nbx, int nq, int x, int y) {
  return (((uint32_t(y) * uint32_t(nbx) + uint32_t(x >> 6)) * uint32_t(nq) << 6) + uint32_t(x & 63)) *
         uint32_t(sizeof(T));
}

template <typename T>
__device__ __forceinline__ T load_at(const T* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// rho^sigma at (x, y), summing the pulled populations in lattice order (the
// same order as the split path's density kernel).
template <typename T, int NC>
__device__ __forceinline__ void pulled_density(const T* __restrict__ fin, const Params<T>& p, int x, int y,
                                               T (&rho)[NC]) {
  using L = Lattice<2>;
  const int xm = wrap_add(x, -1, p.nx), xp = wrap_add(x, 1, p.nx);
  const int ym = wrap_add(y, -1, p.ny), yp = wrap_add(y, 1, p.ny);
  uint32_t off[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const int sx = L::cx(i) > 0 ? xm : (L::cx(i) < 0 ? xp : x);
    const int sy = L::cy(i) > 0 ? ym : (L::cy(i) < 0 ? yp : y);
    off[i] = site_offset<T>(p.nbx, p.nq, sx, sy) + uint32_t(run_slot<L::Q>(i) * kBlockX * sizeof(T));
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    T acc = T(0);
    if (k < p.n) {
#pragma unroll
      for (int i = 0; i < L::Q; ++i) acc += load_at(fin, off[i] + uint32_t(k * L::Q * kBlockX * sizeof(T)));
    }
    rho[k] = acc;
  }
}

// LDS of one tile step.
template <typename T, int NC, int TX, int TY>
struct TileLds {
  T rho[NC][TY + 4][TX + 4];  // rho region: tile + 2
  T h[NC][TY + 2][TX + 2];    // h region:   tile + 1
};

// The whole step for the tile with corner (x0, y0).  Every thread of the
// workgroup calls it (it contains workgroup barriers).
template <typename T, int NC, int TX, int TY, int NT, bool NTSTORE>
__device__ __forceinline__ void tile_step(const T* __restrict__ fin, T* __restrict__ fout, const Params<T>& p,
                                          int x0, int y0, TileLds<T, NC, TX, TY>& lds) {
  using L = Lattice<2>;
  constexpr int Q = L::Q;
  constexpr int HX = TX + 4, HY = TY + 4;  // rho region: tile + 2
  constexpr int GX = TX + 2, GY = TY + 2;  // h region:   tile + 1
  constexpr int RS = NT / TX;              // row stride between a thread's sites
  constexpr int SPT = TY / RS;             // sites per thread
  static_assert(NT % TX == 0 && TY % RS == 0, "tile shape");
  auto& s_rho = lds.rho;
  auto& s_h = lds.h;
  const int nx = p.nx, ny = p.ny, n = p.n;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;

  // ---- A: the tile's own populations, kept in registers -------------------
  T f[SPT][NC][Q];
  bool valid[SPT];
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int x = x0 + tx, y = y0 + ty + k * RS;
    valid[k] = x < nx && y < ny;
    if (valid[k]) {
      const int xm = wrap_add(x, -1, nx), xp = wrap_add(x, 1, nx);
      const int ym = wrap_add(y, -1, ny), yp = wrap_add(y, 1, ny);
      uint32_t off[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int sx = L::cx(i) > 0 ? xm : (L::cx(i) < 0 ? xp : x);
        const int sy = L::cy(i) > 0 ? ym : (L::cy(i) < 0 ? yp : y);
        off[i] = site_offset<T>(p.nbx, p.nq, sx, sy) + uint32_t(run_slot<Q>(i) * kBlockX * sizeof(T));
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          f[k][c][i] = c < n ? load_at(fin, off[i] + uint32_t(c * Q * kBlockX * sizeof(T))) : T(0);
          acc += f[k][c][i];
        }
        s_rho[c][ty + k * RS + 2][tx + 2] = acc;
      }
    }
  }

  // ---- B: density on the ring (and on tile slots outside a ragged box) ----
  const bool full = (x0 + TX <= nx) && (y0 + TY <= ny);
  if (full) {
    constexpr int RING = 4 * HX + 4 * TY;
    for (int idx = threadIdx.x; idx < RING; idx += NT) {
      int px, py;
      if (idx < 2 * HX) {
        py = idx / HX;
        px = idx % HX;
      } else if (idx < 4 * HX) {
        const int j = idx - 2 * HX;
        py = TY + 2 + j / HX;
        px = j % HX;
      } else if (idx < 4 * HX + 2 * TY) {
        const int j = idx - 4 * HX;
        py = 2 + j / 2;
        px = j % 2;
      } else {
        const int j = idx - 4 * HX - 2 * TY;
        py = 2 + j / 2;
        px = TX + 2 + j % 2;
      }
      T r[NC];
      pulled_density<T, NC>(fin, p, wrap_mod(x0 - 2 + px, nx), wrap_mod(y0 - 2 + py, ny), r);
#pragma unroll
      for (int c = 0; c < NC; ++c) s_rho[c][py][px] = r[c];
    }
  } else {
    for (int idx = threadIdx.x; idx < HX * HY; idx += NT) {
      const int px = idx % HX, py = idx / HX;
      const bool inner = px >= 2 && px < TX + 2 && py >= 2 && py < TY + 2 && x0 + px - 2 < nx && y0 + py - 2 < ny;
      if (inner) continue;  // filled in phase A
      T r[NC];
      pulled_density<T, NC>(fin, p, wrap_mod(x0 - 2 + px, nx), wrap_mod(y0 - 2 + py, ny), r);
#pragma unroll
      for (int c = 0; c < NC; ++c) s_rho[c][py][px] = r[c];
    }
  }
  __syncthreads();

  // ---- C: potential h on the tile plus one ring ---------------------------
  for (int idx = threadIdx.x; idx < GX * GY; idx += NT) {
    const int qx = idx % GX, qy = idx / GX;
    const int cx = qx + 1, cy = qy + 1;  // position in the rho region
    T r[NC], lap[NC], mu[NC], h[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      r[c] = c < n ? s_rho[c][cy][cx] : T(1);
      lap[c] = c < n ? lattice_laplacian<2, T>(
                           [&](int i) { return s_rho[c][cy + L::cy(i)][cx + L::cx(i)]; }, r[c])
                     : T(0);
    }
    site_potential<T, NC>(p, r, lap, mu, h);
#pragma unroll
    for (int c = 0; c < NC; ++c) s_h[c][qy][qx] = h[c];
  }
  __syncthreads();

  // ---- D: force, equilibrium, forcing term, collision, store -------------
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    if (!valid[k]) continue;
    const int ly = ty + k * RS;
    const int x = x0 + tx, y = y0 + ly;
    T rs[NC], jx[NC], jy[NC];
    T rt = T(0), ux = T(0), uy = T(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T ax = T(0), ay = T(0);
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        if (L::cx(i)) ax += T(L::cx(i)) * f[k][c][i];
        if (L::cy(i)) ay += T(L::cy(i)) * f[k][c][i];
      }
      jx[c] = ax;
      jy[c] = ay;
      rs[c] = s_rho[c][ly + 2][tx + 2];
      if (c < n) {
        ux += ax;
        uy += ay;
        rt += rs[c];
      }
    }
    const T inv_rt = rcp_(rt);
    ux *= inv_rt;
    uy *= inv_rt;
    const uint32_t own = site_offset<T>(p.nbx, p.nq, x, y);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (c >= n) continue;
      T Ax, Ay, Az;
      lattice_force<2, T>([&](int i) { return s_h[c][ly + 1 + L::cy(i)][tx + 1 + L::cx(i)]; },
                          [&](int i) { return s_rho[c][ly + 2 + L::cy(i)][tx + 2 + L::cx(i)]; }, rs[c], p, Ax,
                          Ay, Az);
      const T inv_rs = rcp_(rs[c]);
      collide<2, T>(f[k][c], rs[c], ux, uy, T(0), Ax, Ay, Az, jx[c] * inv_rs, jy[c] * inv_rs, T(0), p.inv_tau);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        T* dst = reinterpret_cast<T*>(reinterpret_cast<char*>(fout) + own +
                                      uint32_t((c * Q + run_slot<Q>(i)) * kBlockX * sizeof(T)));
        if constexpr (NTSTORE)
          __builtin_nontemporal_store(f[k][c][i], dst);
        else
          *dst = f[k][c][i];
      }
    }
  }
}

template <typename T, int NC, int TX, int TY, int NT, bool NTSTORE>
__global__ void __launch_bounds__(NT) k_fused_d2q9(const T* __restrict__ fin, T* __restrict__ fout, Params<T> p,
                                                   int nbx, int ntiles, int tiles_per_xcd, int xcd_remap) {
  __shared__ TileLds<T, NC, TX, TY> lds;
  // XCD-aware tile order: workgroup b runs on XCD b % 8; give XCD c the
  // contiguous tile range [c * tiles_per_xcd, (c + 1) * tiles_per_xcd).
  const int b = blockIdx.x;
  const int t = xcd_remap ? (b % kXcds) * tiles_per_xcd + b / kXcds : b;
  if (t >= ntiles) return;
  tile_step<T, NC, TX, TY, NT, NTSTORE>(fin, fout, p, (t % nbx) * TX, (t / nbx) * TY, lds);
}

// ---------------------------------------------------------- batched ----
// Persistent step of many independent lattices in one launch.  The host
// owns the slot table (parameters, population copies, tile ranges, target
// step) and the map from work item to table entry; the device owns the step
// counters.  A slot whose counter has reached its target is skipped, so one
// captured sequence of launches stays valid while slots join and leave; the
// population copy read at step t is f[t & 1].  Work items (slot, tile) are
// numbered consecutively over the live slots; XCD c (dispatch is round
// robin) takes the contiguous range [c * per_xcd, (c + 1) * per_xcd), its
// workgroups striding through it, so that the halo rows of neighbouring
// tiles stay in that XCD's L2.
template <typename T, int NC, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_batch_d2q9(const BatchSlot<T>* __restrict__ slots,
                                                   const long long* __restrict__ t_now,
                                                   const BatchHeader* __restrict__ hdr,
                                                   const int* __restrict__ item_slot) {
  __shared__ TileLds<T, NC, TX, TY> lds;
  const int items = hdr->items;
  const int groups = gridDim.x / kXcds;  // workgroups per XCD (the grid is a multiple of 8)
  const int per_xcd = (items + kXcds - 1) / kXcds;
  const int xcd = blockIdx.x % kXcds, g = blockIdx.x / kXcds;
  for (int j = g; j < per_xcd; j += groups) {
    const int w = xcd * per_xcd + j;
    if (w >= items) break;
    const BatchSlot<T>& sl = slots[item_slot[w]];
    const long long t = t_now[sl.id];
    if (t >= sl.t_end) continue;  // uniform: the whole workgroup skips
    const int tile = w - sl.first_item;
    const int x0 = (tile % sl.tiles_x) * TX, y0 = (tile / sl.tiles_x) * TY;
    tile_step<T, NC, TX, TY, NT, true>(static_cast<const T*>(sl.f[t & 1]), static_cast<T*>(sl.f[(t + 1) & 1]),
                                       sl.p, x0, y0, lds);
    __syncthreads();  // the next tile reuses the LDS
  }
}

// Counters of the slots the step launch before stepped: t += 1 below target.
template <typename T>
__global__ void k_batch_advance(const BatchSlot<T>* __restrict__ slots, long long* __restrict__ t_now,
                                const BatchHeader* __restrict__ hdr) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= hdr->nslots) return;
  const int id = slots[s].id;
  if (t_now[id] < slots[s].t_end) t_now[id] += 1;
}

template <typename T, int NC, int TX, int TY, int NT>
static void batch_step_launch(const void* slots, const long long* t_now, const BatchHeader* hdr,
                              const int* item_slot, int grid, hipStream_t s) {
  k_batch_d2q9<T, NC, TX, TY, NT><<<grid, NT, 0, s>>>(static_cast<const BatchSlot<T>*>(slots), t_now, hdr,
                                                       item_slot);
}

template <typename T>
static void batch_advance_launch(const void* slots, long long* t_now, const BatchHeader* hdr, int max_slots,
                                 hipStream_t s) {
  k_batch_advance<T><<<(max_slots + 255) / 256, 256, 0, s>>>(static_cast<const BatchSlot<T>*>(slots), t_now, hdr);
}

template <typename T, int NC, int TX, int TY, int NT>
static constexpr BatchKernel batch_kernel() {
  return BatchKernel{TX, TY, NT, batch_step_launch<T, NC, TX, TY, NT>, batch_advance_launch<T>};
}

// Candidate tile shapes for the autotuner, per precision and component
// bound: FP32 keeps SPT * NC * 9 populations per thread in registers, FP64
// twice the bytes, so FP64 and large NC get the shorter tiles.
template <typename T, int NC>
static const BatchKernel* batch_list(int* n) {
  if constexpr (sizeof(T) == 4 && NC <= 3) {
    static const BatchKernel k[] = {batch_kernel<T, NC, 64, 16, 256>(), batch_kernel<T, NC, 64, 8, 256>(),
                                    batch_kernel<T, NC, 64, 4, 256>(),  batch_kernel<T, NC, 128, 8, 256>(),
                                    batch_kernel<T, NC, 32, 16, 256>(), batch_kernel<T, NC, 32, 8, 256>()};
    *n = int(sizeof(k) / sizeof(k[0]));
    return k;
  } else {
    static const BatchKernel k[] = {batch_kernel<T, NC, 64, 8, 256>(), batch_kernel<T, NC, 64, 4, 256>(),
                                    batch_kernel<T, NC, 32, 8, 256>()};
    *n = int(sizeof(k) / sizeof(k[0]));
    return k;
  }
}

const BatchKernel* batch_kernels(int storage, int max_comp, int* n) {
  *n = 0;
  if (storage == 1) {
    switch (max_comp) {
      case 1: return batch_list<float, 1>(n);
      case 2: return batch_list<float, 2>(n);
      case 3: return batch_list<float, 3>(n);
      case 4: return batch_list<float, 4>(n);
      default: return nullptr;
    }
  }
  if (storage == 0) {
    switch (max_comp) {
      case 1: return batch_list<double, 1>(n);
      case 2: return batch_list<double, 2>(n);
      case 3: return batch_list<double, 3>(n);
      case 4: return batch_list<double, 4>(n);
      default: return nullptr;
    }
  }
  return nullptr;
}

// ------------------------------------------------------------ dispatch ----
template <typename T, int NC, int TX, int TY, int NT = 256, bool NTSTORE = true>
static void launch_tile(const Params<T>& p, const T* fin, T* fout, hipStream_t stream, bool remap = true) {
  const int nbx = (p.nx + TX - 1) / TX;
  const int nby = (p.ny + TY - 1) / TY;
  const int ntiles = nbx * nby;
  const int per_xcd = (ntiles + kXcds - 1) / kXcds;
  const int grid = remap ? per_xcd * kXcds : ntiles;
  k_fused_d2q9<T, NC, TX, TY, NT, NTSTORE><<<grid, NT, 0, stream>>>(fin, fout, p, nbx, ntiles, per_xcd, remap);
}

template <typename T, int NC, int TX, int TY>
static void launch_fused(const Ctx& c, const void* fin, void* fout) {
  launch_tile<T, NC, TX, TY>(c.params<T>(), static_cast<const T*>(fin), static_cast<T*>(fout), c.stream);
}

// Tile per precision and component count: registers hold SPT * N * 9
// populations per thread and LDS holds N rho and N h tiles.
template <typename T, int NC>
static FusedStepFn pick() {
  if constexpr (sizeof(T) == 4) {
    if constexpr (NC <= 3) return launch_fused<T, NC, 64, 16>;
    else if constexpr (NC <= 5) return launch_fused<T, NC, 64, 8>;
    else return launch_fused<T, NC, 64, 4>;
  } else {
    if constexpr (NC <= 2) return launch_fused<T, NC, 64, 8>;
    else return launch_fused<T, NC, 64, 4>;
  }
}

template <typename T>
static FusedStepFn pick_n(int n) {
  switch (n) {
    case 1: return pick<T, 1>();
    case 2: return pick<T, 2>();
    case 3: return pick<T, 3>();
    case 4: return pick<T, 4>();
    case 5: return pick<T, 5>();
    case 6: return pick<T, 6>();
    case 7: return pick<T, 7>();
    case 8: return pick<T, 8>();
    default: return nullptr;
  }
}

FusedStepFn fused_step_for(int lattice, int storage, int n_comp) {
  if (lattice != 2) return nullptr;  // slot-count limit checked by the caller
  if (storage == 0) return pick_n<double>(n_comp);
  if (storage == 1) return pick_n<float>(n_comp);
  return nullptr;  // shifted FP16 storage: split and sweep paths only
}

}  // namespace lbm
