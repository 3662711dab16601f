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
// The kernel is templated on the storage codec (storage.hpp): FP64, FP32,
// or shifted FP16 (decoded on load against the references of the source
// sites, the density from the exact pulled total, encoded on store against
// the site's new reference).  Boxes closed by walls take a separate
// instantiation: bounce-back in the pull, mirrored layers beyond a wall in
// the density and potential rings (the split path's values, bit for bit).  No MFMA: the step is a bandwidth-bound stencil, not a
// contraction.
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

// 32-bit byte offset of the block that holds site (x, y) (the block layout
// of storage.hpp: n components of kComp bytes per 64-site block).  The host
// only takes this path when one population copy is smaller than 4 GiB, so
// that every access is a uniform 64-bit base plus a 32-bit per-lane offset.
template <class S>
__device__ __forceinline__ uint32_t block_off(const Params<typename S::T>& p, int x, int y) {
  return (uint32_t(y) * uint32_t(p.nbx) + uint32_t(x >> 6)) * uint32_t(p.n) * BlockLayout<S, 9>::kComp;
}

// Loads and stores of population slots through the global address space.
// The batched kernel reads its population pointers from the slot table,
// where the compiler cannot tell their address space and would otherwise
// emit flat accesses (which also count against the LDS counter).
using GChar = __attribute__((address_space(1))) char;

template <class S>
__device__ __forceinline__ typename S::T gload_slot(const void* base, uint32_t off, int i) {
  using T = typename S::T;
  const GChar* b = (const GChar*)base + off;
  if (i == 0) return T(*(const __attribute__((address_space(1))) typename S::Rest*)b);
  return T(*(const __attribute__((address_space(1))) typename S::Move*)b);
}

// FP16 value (moving slot or reference of the shifted codec) and FP32 value
// at a byte offset.
__device__ __forceinline__ _Float16 gload_half(const void* base, uint32_t off) {
  return *(const __attribute__((address_space(1))) _Float16*)((const GChar*)base + off);
}
__device__ __forceinline__ float gload_f32(const void* base, uint32_t off) {
  return *(const __attribute__((address_space(1))) float*)((const GChar*)base + off);
}

template <bool NTSTORE, typename V>
__device__ __forceinline__ void gstore(void* base, uint32_t off, V v) {
  __attribute__((address_space(1))) V* d = (__attribute__((address_space(1))) V*)((GChar*)base + off);
  if constexpr (NTSTORE)
    __builtin_nontemporal_store(v, d);
  else
    *d = v;
}

// Coordinate of the site whose values stand at coordinate v of an axis of n
// layers: periodic, or, on an axis closed by walls, the mirror image of the
// layer next to the wall for the first two layers beyond it (zero normal
// gradient of the stencils' fields, as on the split path); positions further
// out (only in ragged tiles, where no site reads them) wrap, which keeps
// every access inside the box.
__device__ __forceinline__ int axis_site(int v, int n, bool wall) {
  if (wall) v = v < 0 ? -1 - v : (v >= n ? 2 * n - 1 - v : v);
  return wrap_mod(v, n);
}

// Byte offsets, without the component part, of the nine slots pulled into
// site (x, y) (slot i of the site r - v_i) and, for the shifted codec, of
// the references of those sites.  Where r - v_i lies beyond a wall the slot
// is -v_i of r itself (half-way bounce-back); its offset then also carries
// the distance from run i to run -v_i (the same for every component), so
// that adding run(c, i) lands on run(c, -v_i).
template <class S, bool W>
__device__ __forceinline__ void pull_offsets(const Params<typename S::T>& p, int x, int y, uint32_t (&off)[9],
                                             uint32_t (&roff)[9]) {
  using L = Lattice<2>;
  using B = BlockLayout<S, 9>;
  const int xm = wrap_add(x, -1, p.nx), xp = wrap_add(x, 1, p.nx);
  const int ym = wrap_add(y, -1, p.ny), yp = wrap_add(y, 1, p.ny);
  if constexpr (!W) {  // periodic box
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      const int sx = L::cx(i) > 0 ? xm : (L::cx(i) < 0 ? xp : x);
      const int sy = L::cy(i) > 0 ? ym : (L::cy(i) < 0 ? yp : y);
      const uint32_t blk = block_off<S>(p, sx, sy);
      off[i] = blk + B::in_run(i, sx);
      roff[i] = blk + B::in_ref(sx);
    }
  } else {
    const bool wx = p.walls & 1, wy = p.walls & 2;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      int sx = L::cx(i) > 0 ? xm : (L::cx(i) < 0 ? xp : x);
      int sy = L::cy(i) > 0 ? ym : (L::cy(i) < 0 ? yp : y);
      uint32_t hop = 0;
      if (i > 0) {
        const int ux = x - L::cx(i), uy = y - L::cy(i);
        const bool beyond = (wx && (ux < 0 || ux >= p.nx)) || (wy && (uy < 0 || uy >= p.ny));
        sx = beyond ? x : sx;
        sy = beyond ? y : sy;
        hop = beyond ? B::run(0, L::opp(i)) - B::run(0, i) : 0u;
      }
      const uint32_t blk = block_off<S>(p, sx, sy);
      off[i] = blk + B::in_run(i, sx) + hop;
      roff[i] = blk + B::in_ref(sx);
    }
  }
}

// Pulled populations of component c at a site from its offsets: decoded
// values and their running sum (take_slot, take_shifted).
template <class S>
__device__ __forceinline__ void pull_component(const void* __restrict__ fin, const Params<typename S::T>& p, int c,
                                               const uint32_t (&off)[9], const uint32_t (&roff)[9],
                                               typename S::T (&f)[9], typename S::T& sum) {
  using T = typename S::T;
  using B = BlockLayout<S, 9>;
  sum = T(0);
  if constexpr (S::kShift) {
    float rest = 0.f;
    _Float16 d[9], h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (i == 0)
        rest = gload_f32(fin, off[0] + B::run(c, 0));
      else
        d[i] = gload_half(fin, off[i] + B::run(c, i));
      h[i] = gload_half(fin, roff[i] + B::ref(c));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) take_shifted<2>(i, i == 0 ? _Float16(0) : d[i], rest, h[i], p.sh.scale[c], p.sh.one, sum, f[i]);
  } else {
    T raw[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) raw[i] = gload_slot<S>(fin, off[i] + B::run(c, i), i);
#pragma unroll
    for (int i = 0; i < 9; ++i) take_slot<S, 2>(i, raw[i], sum, f[i]);
  }
}

// rho^sigma at (x, y) from the pulled slots: the sum of the decoded
// populations in lattice order, or s times the exact pulled total for the
// shifted codec (the same values as the split path's density kernel).
template <class S, int NC, bool W>
__device__ __forceinline__ void pulled_density(const void* __restrict__ fin, const Params<typename S::T>& p, int x,
                                               int y, typename S::T (&rho)[NC]) {
  using T = typename S::T;
  uint32_t off[9], roff[9];
  pull_offsets<S, W>(p, x, y, off, roff);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    T v[9], sum = T(0);
    if (k < p.n) {
      pull_component<S>(fin, p, k, off, roff, v, sum);
      rho[k] = site_density<S>(sum, p.sh.scale[k]);
    } else {
      rho[k] = T(0);
    }
  }
}

// LDS of one tile step.
template <typename T, int NC, int TX, int TY>
struct TileLds {
  T rho[NC][TY + 4][TX + 4];  // rho region: tile + 2
  T h[NC][TY + 2][TX + 2];    // h region:   tile + 1
};

// The whole step for the tile with corner (x0, y0).  Every thread of the
// workgroup calls it (it contains workgroup barriers).  W: the box has walls
// (p.walls != 0; a separate instantiation keeps the periodic step free of
// the wall logic).
template <class S, int NC, int TX, int TY, int NT, bool NTSTORE, bool W>
__device__ __forceinline__ void tile_step(const void* __restrict__ fin, void* __restrict__ fout,
                                          const Params<typename S::T>& p, int x0, int y0,
                                          TileLds<typename S::T, NC, TX, TY>& lds) {
  using T = typename S::T;
  using B = BlockLayout<S, 9>;
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
  // (decoded; the shifted codec also keeps each site's ledger)
  T f[SPT][NC][Q];
  T led[SPT][NC];
  bool valid[SPT];
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int x = x0 + tx, y = y0 + ty + k * RS;
    valid[k] = x < nx && y < ny;
    if (valid[k]) {
      uint32_t off[Q], roff[Q];
      pull_offsets<S, W>(p, x, y, off, roff);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        // one uniform branch per component, so that its loads are issued
        // together
        T l = T(0);
        if (c < n) {
          pull_component<S>(fin, p, c, off, roff, f[k][c], l);
        } else {
#pragma unroll
          for (int i = 0; i < Q; ++i) f[k][c][i] = T(0);
        }
        led[k][c] = l;
        s_rho[c][ty + k * RS + 2][tx + 2] = c < n ? site_density<S>(l, p.sh.scale[c]) : T(0);
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
      pulled_density<S, NC, W>(fin, p, axis_site(x0 - 2 + px, nx, W && (p.walls & 1)),
                               axis_site(y0 - 2 + py, ny, W && (p.walls & 2)),
                            r);
#pragma unroll
      for (int c = 0; c < NC; ++c) s_rho[c][py][px] = r[c];
    }
  } else {
    for (int idx = threadIdx.x; idx < HX * HY; idx += NT) {
      const int px = idx % HX, py = idx / HX;
      const bool inner = px >= 2 && px < TX + 2 && py >= 2 && py < TY + 2 && x0 + px - 2 < nx && y0 + py - 2 < ny;
      if (inner) continue;  // filled in phase A
      T r[NC];
      pulled_density<S, NC, W>(fin, p, axis_site(x0 - 2 + px, nx, W && (p.walls & 1)),
                               axis_site(y0 - 2 + py, ny, W && (p.walls & 2)),
                            r);
#pragma unroll
      for (int c = 0; c < NC; ++c) s_rho[c][py][px] = r[c];
    }
  }
  __syncthreads();

  // ---- C: potential h on the tile plus one ring ---------------------------
  // (a position one layer beyond a wall takes h of the layer next to it,
  // computed there from the same neighbours as on the split path)
  for (int idx = threadIdx.x; idx < GX * GY; idx += NT) {
    const int qx = idx % GX, qy = idx / GX;
    int cx = qx + 1, cy = qy + 1;  // position in the rho region
    if (W && (p.walls & 1)) {
      const int X = x0 - 1 + qx;
      cx = X == -1 ? cx + 1 : (X == nx ? cx - 1 : cx);
    }
    if (W && (p.walls & 2)) {
      const int Y = y0 - 1 + qy;
      cy = Y == -1 ? cy + 1 : (Y == ny ? cy - 1 : cy);
    }
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
    const uint32_t own = block_off<S>(p, x, y);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (c >= n) continue;
      T Ax, Ay, Az;
      lattice_force<2, T>([&](int i) { return s_h[c][ly + 1 + L::cy(i)][tx + 1 + L::cx(i)]; },
                          [&](int i) { return s_rho[c][ly + 2 + L::cy(i)][tx + 2 + L::cx(i)]; }, rs[c], p, Ax,
                          Ay, Az);
      const T inv_rs = rcp_(rs[c]);
      collide<2, T>(f[k][c], rs[c], ux, uy, T(0), Ax, Ay, Az, jx[c] * inv_rs, jy[c] * inv_rs, T(0), p.inv_tau);
      if constexpr (S::kShift) {
        // the site's new reference, the FP16 deviations of the moving
        // populations, and the rest of the ledger
        const _Float16 h = new_ref(led[k][c]);
        _Float16 d[Q];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          d[i] = encode_move<2>(i, f[k][c][i], p.sh.inv_scale[c], float(h));
          gstore<NTSTORE>(fout, own + B::run(c, i) + B::in_run(i, x), d[i]);
        }
        gstore<NTSTORE>(fout, own + B::ref(c) + B::in_ref(x), h);
        gstore<NTSTORE>(fout, own + B::run(c, 0) + B::in_run(0, x), ledger_rest<Q>(led[k][c], float(h), d, p.sh.minus_one));
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) gstore<NTSTORE>(fout, own + B::run(c, i) + B::in_run(i, x), f[k][c][i]);
      }
    }
  }
}

template <class S, int NC, int TX, int TY, int NT, bool NTSTORE, bool W>
__global__ void __launch_bounds__(NT) k_fused_d2q9(const void* __restrict__ fin, void* __restrict__ fout,
                                                   Params<typename S::T> p, int nbx, int ntiles, int tiles_per_xcd,
                                                   int xcd_remap) {
  __shared__ TileLds<typename S::T, NC, TX, TY> lds;
  // XCD-aware tile order: workgroup b runs on XCD b % 8; give XCD c the
  // contiguous tile range [c * tiles_per_xcd, (c + 1) * tiles_per_xcd).
  const int b = blockIdx.x;
  const int t = xcd_remap ? (b % kXcds) * tiles_per_xcd + b / kXcds : b;
  if (t >= ntiles) return;
  tile_step<S, NC, TX, TY, NT, NTSTORE, W>(fin, fout, p, (t % nbx) * TX, (t / nbx) * TY, lds);
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
template <class S, int NC, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_batch_d2q9(const BatchSlot<typename S::T>* __restrict__ slots,
                                                   const long long* __restrict__ t_now,
                                                   const BatchHeader* __restrict__ hdr,
                                                   const int* __restrict__ item_slot) {
  using T = typename S::T;
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
    tile_step<S, NC, TX, TY, NT, true, false>(sl.f[t & 1], sl.f[(t + 1) & 1], sl.p, x0, y0, lds);  // periodic runs
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

template <class S, int NC, int TX, int TY, int NT>
static void batch_step_launch(const void* slots, const long long* t_now, const BatchHeader* hdr,
                              const int* item_slot, int grid, hipStream_t s) {
  k_batch_d2q9<S, NC, TX, TY, NT><<<grid, NT, 0, s>>>(static_cast<const BatchSlot<typename S::T>*>(slots), t_now,
                                                       hdr, item_slot);
}

template <typename T>
static void batch_advance_launch(const void* slots, long long* t_now, const BatchHeader* hdr, int max_slots,
                                 hipStream_t s) {
  k_batch_advance<T><<<(max_slots + 255) / 256, 256, 0, s>>>(static_cast<const BatchSlot<T>*>(slots), t_now, hdr);
}

template <class S, int NC, int TX, int TY, int NT>
static constexpr BatchKernel batch_kernel() {
  return BatchKernel{TX, TY, NT, batch_step_launch<S, NC, TX, TY, NT>, batch_advance_launch<typename S::T>};
}

// Candidate tile shapes for the autotuner, per precision and component
// bound: FP32 (and the shifted codec, decoded to FP32) keeps SPT * NC * 9
// populations per thread in registers, FP64 twice the bytes, so FP64 and
// large NC get the shorter tiles.
template <class S, int NC>
static const BatchKernel* batch_list(int* n) {
  if constexpr (sizeof(typename S::T) == 4 && NC <= 3) {
    static const BatchKernel k[] = {batch_kernel<S, NC, 64, 16, 256>(), batch_kernel<S, NC, 64, 8, 256>(),
                                    batch_kernel<S, NC, 64, 4, 256>(),  batch_kernel<S, NC, 128, 8, 256>(),
                                    batch_kernel<S, NC, 32, 16, 256>(), batch_kernel<S, NC, 32, 8, 256>()};
    *n = int(sizeof(k) / sizeof(k[0]));
    return k;
  } else {
    static const BatchKernel k[] = {batch_kernel<S, NC, 64, 8, 256>(), batch_kernel<S, NC, 64, 4, 256>(),
                                    batch_kernel<S, NC, 32, 8, 256>()};
    *n = int(sizeof(k) / sizeof(k[0]));
    return k;
  }
}

template <class S>
static const BatchKernel* batch_for_n(int max_comp, int* n) {
  switch (max_comp) {
    case 1: return batch_list<S, 1>(n);
    case 2: return batch_list<S, 2>(n);
    case 3: return batch_list<S, 3>(n);
    case 4: return batch_list<S, 4>(n);
    default: return nullptr;
  }
}

const BatchKernel* batch_kernels(int storage, int max_comp, int* n) {
  *n = 0;
  if (storage == StoreF64::kId) return batch_for_n<StoreF64>(max_comp, n);
  if (storage == StoreF32::kId) return batch_for_n<StoreF32>(max_comp, n);
  if (storage == StoreF16S::kId) return batch_for_n<StoreF16S>(max_comp, n);
  return nullptr;
}

// ------------------------------------------------------------ dispatch ----
template <class S, int NC, int TX, int TY, int NT = 256, bool NTSTORE = true>
static void launch_tile(const Params<typename S::T>& p, const void* fin, void* fout, hipStream_t stream,
                        bool remap = true) {
  const int nbx = (p.nx + TX - 1) / TX;
  const int nby = (p.ny + TY - 1) / TY;
  const int ntiles = nbx * nby;
  const int per_xcd = (ntiles + kXcds - 1) / kXcds;
  const int grid = remap ? per_xcd * kXcds : ntiles;
  if (p.walls)
    k_fused_d2q9<S, NC, TX, TY, NT, NTSTORE, true><<<grid, NT, 0, stream>>>(fin, fout, p, nbx, ntiles, per_xcd, remap);
  else
    k_fused_d2q9<S, NC, TX, TY, NT, NTSTORE, false><<<grid, NT, 0, stream>>>(fin, fout, p, nbx, ntiles, per_xcd,
                                                                            remap);
}

template <class S, int NC, int TX, int TY>
static void launch_fused(const Ctx& c, const void* fin, void* fout) {
  launch_tile<S, NC, TX, TY>(c.params<typename S::T>(), fin, fout, c.stream);
}

// Tile per precision and component count: registers hold SPT * N * 9
// populations per thread (decoded, so the shifted codec counts as FP32) and
// LDS holds N rho and N h tiles.
template <class S, int NC>
static FusedStepFn pick() {
  if constexpr (sizeof(typename S::T) == 4) {
    // (the shifted codec also keeps a ledger per site and component: at
    // N = 5 on 64x8 tiles the register pressure serialises the ring loads)
    constexpr int kMid = S::kShift ? 4 : 5;
    if constexpr (NC <= 3) return launch_fused<S, NC, 64, 16>;
    else if constexpr (NC <= kMid) return launch_fused<S, NC, 64, 8>;
    else return launch_fused<S, NC, 64, 4>;
  } else {
    if constexpr (NC <= 2) return launch_fused<S, NC, 64, 8>;
    else return launch_fused<S, NC, 64, 4>;
  }
}

template <class S>
static FusedStepFn pick_n(int n) {
  switch (n) {
    case 1: return pick<S, 1>();
    case 2: return pick<S, 2>();
    case 3: return pick<S, 3>();
    case 4: return pick<S, 4>();
    case 5: return pick<S, 5>();
    case 6: return pick<S, 6>();
    case 7: return pick<S, 7>();
    case 8: return pick<S, 8>();
    default: return nullptr;
  }
}

FusedStepFn fused_step_for(int lattice, int storage, int n_comp) {
  if (lattice != 2) return nullptr;  // slot-count limit checked by the caller
  if (storage == StoreF64::kId) return pick_n<StoreF64>(n_comp);
  if (storage == StoreF32::kId) return pick_n<StoreF32>(n_comp);
  if (storage == StoreF16S::kId) return pick_n<StoreF16S>(n_comp);
  return nullptr;
}

}  // namespace lbm
