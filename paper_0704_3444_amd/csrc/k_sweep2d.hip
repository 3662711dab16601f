// Strip-sweep D2Q9 step: one launch per time step, every population read
// once and written once, with almost no halo re-reads.
//
// A workgroup of four waves owns a strip of 64 columns (one 64-site block of
// the population layout) and a segment of rows, which it sweeps from top to
// bottom.  Wave w handles the rows y = w (mod 4) of the segment.  One round
// advances four rows; per wave:
//   1. wait for the row it staged one round earlier, take its pulled
//      populations into registers and write its densities (and the halo
//      columns') into the LDS ring of densities;
//   2. stage the populations pulled into its density row of the next round
//      in the same LDS slot with direct global-to-LDS loads: per component
//      the three runs that row pulls from each source row are one
//      contiguous, aligned piece of that row's block (the block layout
//      groups the runs by v_y), three 16-byte-per-lane loads per component,
//      plus, for every run, the aligned 16 bytes at the end of the left
//      neighbour's run and at the start of the right neighbour's (the x
//      shift of lanes 0 and 63 and the four density-halo columns read
//      three columns on either side);
//   3. (barrier) chemical potentials and the potential h of its row into an
//      LDS ring (wave 0 also the eight edge columns of the four rows);
//   4. (barrier) force, equilibrium, forcing term and collision of the row
//      it took one round earlier; non-temporal stores in place (streaming
//      happens through the next step's pull).
// Staged rows are private to their wave, so only the two rings need the
// workgroup barriers; the loads in flight hold no registers.  The compiler
// does not track direct loads into LDS, so the wave waits for its own
// staging with an explicit vmcnt: one counter covers loads and stores and
// retires them in issue order, so the wait names how many operations issued
// after the staging may stay in flight (the stores of the round before).  Workgroups
// are banded per XCD so that neighbouring strips share L2.
//
// The kernel is templated on the storage codec (storage.hpp): FP32, or
// shifted FP16 (decoded when the row is taken from LDS).
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"
#include "physics.hpp"
#include "storage.hpp"

namespace lbm {
namespace sweep {

constexpr int kXcds = 8;
constexpr int kRhoRing = 16;  // rows of rho in LDS: 9 live, and a wave one round ahead writes 12 rows further
constexpr int kHRing = 8;     // rows of h in LDS (8 live; written only between barriers)
constexpr int kW = 64;        // strip width = block width = wave size
constexpr int kRW = kW + 4;   // rho row: columns x0 - 2 .. x0 + 65
constexpr int kHW = kW + 2;   // h row:   columns x0 - 1 .. x0 + 64

__device__ __forceinline__ int wrap_mod(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// s_waitcnt vmcnt(N), the other counters untouched, as a compiler memory
// barrier: the LDS written by the direct loads is read only after it.
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Workgroup barrier that publishes this wave's LDS writes without waiting
// for its global loads in flight.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Staged row: every run that a row pulls, in LDS as one padded segment
// [16 bytes of the left neighbour block's run | the 64 slots of the row's
// own block column | 16 bytes of the right neighbour block's run], so that
// column col (-16/e .. 63 + 16/e, e the slot size) of the run sits at
// segment + 16 + col e and the edge lanes need no selects.  Segments are
// grouped by source row (v_y = 0: the row itself; +1: the row above; -1:
// the row below), and within a group by component, in the block's run order:
// v_y = 0 holds runs 0, 1, 3, v_y = +1 runs 2, 5, 6, v_y = -1 runs 4, 7, 8;
// for the shifted codec each group also holds the reference run of its
// source row (after the component's runs).  The staged row is filled by
// kLoads direct loads of 16 bytes per lane over its consecutive 16-byte
// chunks, every lane active: the lanes beyond the last chunk read a valid
// address and write into the padding after it.  (With the last loads issued
// only by the lanes that have a chunk, the compiler had merged a partial
// load with the next one under divergent control flow and taken one lane's
// LDS destination for both.)  Only a load that straddles two groups selects
// its row part per lane.
template <class S, int NC>
struct Staged {
  using B = BlockLayout<S, 9>;
  using L = Lattice<2>;
  static constexpr int kRunsPerGroup = S::kShift ? 4 : 3;  // three runs (+ the reference run)
  // velocity of run k of group g (k == 3: the reference run)
  static constexpr int vel(int g, int k) {
    constexpr int v[3][3] = {{0, 1, 3}, {2, 5, 6}, {4, 7, 8}};
    return v[g][k];
  }
  static constexpr uint32_t elem(int g, int k) { return k == 3 ? B::kRef : (vel(g, k) == 0 ? B::kRest : B::kMove); }
  static constexpr uint32_t seg_bytes(int g, int k) { return 32u + uint32_t(kW) * elem(g, k); }
  static constexpr uint32_t comp_bytes(int g) {
    uint32_t n = 0;
    for (int k = 0; k < kRunsPerGroup; ++k) n += seg_bytes(g, k);
    return n;
  }
  static constexpr uint32_t group_bytes(int g) { return NC * comp_bytes(g); }
  static constexpr uint32_t group_off(int g) { return g == 0 ? 0u : (g == 1 ? group_bytes(0) : group_bytes(0) + group_bytes(1)); }
  // LDS byte offset of segment (g, c, k)
  static constexpr uint32_t seg(int g, int c, int k) {
    uint32_t o = group_off(g) + uint32_t(c) * comp_bytes(g);
    for (int q = 0; q < k; ++q) o += seg_bytes(g, q);
    return o;
  }
  static constexpr int group_of(int i) { return L::cy(i) == 0 ? 0 : (L::cy(i) > 0 ? 1 : 2); }
  static constexpr int slot_of(int i) {
    const int g = group_of(i);
    return vel(g, 0) == i ? 0 : (vel(g, 1) == i ? 1 : 2);
  }
  // LDS byte offset of column 0 of run i of component c, of the reference run
  // of component c in the source row dy
  static constexpr uint32_t run0(int c, int i) { return seg(group_of(i), c, slot_of(i)) + 16u; }
  static constexpr uint32_t ref0(int c, int dy) { return seg(dy == 0 ? 0 : (dy > 0 ? 1 : 2), c, 3) + 16u; }
  static constexpr int chunks(int g) { return int(group_bytes(g) / 16); }
  static constexpr int kChunks = chunks(0) + chunks(1) + chunks(2);
  static constexpr int kLoads = (kChunks + 63) / 64;  // direct loads per staged row
  static constexpr uint32_t kBytes = 1024u * uint32_t(kLoads);  // chunks and padding
  static constexpr int kStores = (S::kShift ? 10 : 9) * NC;  // stores per collided row
  static_assert(group_bytes(0) % 16 == 0 && group_bytes(1) % 16 == 0, "segments aligned");
  static_assert(kStores < 64, "vmcnt range");
  // a bounced run of group 1 or 2 is read from the same slot of the other
  static_assert(vel(1, 0) == L::opp(vel(2, 0)) && vel(1, 1) == L::opp(vel(2, 1)) && vel(1, 2) == L::opp(vel(2, 2)),
                "opposite runs share their slot");
};

// Per-lane column parts of the staging loads, which do not change along the
// sweep: load j reads, in lane l, chunk 64 j + l of the staged row: the byte
// offset, less the row part, of that 16-byte chunk in the left neighbour
// block, the strip's own block or the right neighbour block (lanes past the
// last chunk: the strip's own block).
template <class S, int NC>
struct Gather {
  uint32_t col[Staged<S, NC>::kLoads];
  // boxes with walls on y: the distance from the chunk's run to the opposite
  // run of the other vertical group (moving runs of the groups v_y = +1 and
  // -1; 0 elsewhere), which a row next to a wall reads instead (bounce-back)
  uint32_t adj[Staged<S, NC>::kLoads];
};

template <class S, int NC>
__device__ __forceinline__ Gather<S, NC> make_gather(const Params<float>& p, int lane, int x0) {
  using B = BlockLayout<S, 9>;
  using G = Staged<S, NC>;
  constexpr uint32_t comp = NC * B::kComp;
  const uint32_t own = uint32_t(x0 >> 6) * comp;
  const uint32_t left = uint32_t(wrap_add(x0, -1, p.nx) >> 6) * comp;
  const uint32_t right = uint32_t(wrap_add(x0 + kW - 1, 1, p.nx) >> 6) * comp;
  Gather<S, NC> gat;
#pragma unroll
  for (int j = 0; j < G::kLoads; ++j) {
    const int ch = j * 64 + lane;
    const int g = ch < G::chunks(0) ? 0 : (ch < G::chunks(0) + G::chunks(1) ? 1 : 2);
    const int first = g == 0 ? 0 : (g == 1 ? G::chunks(0) : G::chunks(0) + G::chunks(1));
    gat.adj[j] = 0;
    if (ch >= G::kChunks) {
      gat.col[j] = own;
      continue;
    }
    const uint32_t byte = uint32_t(ch - first) * 16u;  // within the group
    // segment of the chunk: component, run slot and position in it
    const uint32_t cb = G::comp_bytes(g);
    const int c = int(byte / cb);
    uint32_t in = byte - uint32_t(c) * cb;
    int k = 0;
#pragma unroll
    for (int q = 0; q < G::kRunsPerGroup - 1; ++q)
      if (in >= G::seg_bytes(g, k)) {
        in -= G::seg_bytes(g, k);
        ++k;
      }
    const uint32_t run = k == 3 ? B::ref(c) : B::run(c, G::vel(g, k));
    const uint32_t len = uint32_t(kW) * G::elem(g, k);  // bytes of the run in a block
    uint32_t off;
    if (in < 16u)
      off = left + run + len - 16u;  // left neighbour's last 16 bytes
    else if (in < 16u + len)
      off = own + run + (in - 16u);
    else
      off = right + run;  // right neighbour's first 16 bytes
    gat.col[j] = off;
    if (g != 0 && k < 3) gat.adj[j] = B::run(c, G::vel(3 - g, k)) - B::run(c, G::vel(g, k));
  }
  return gat;
}

// Stage the populations pulled into row r (wave-uniform) of the strip into
// the LDS slot `dst` (Staged layout) with exactly Staged::kLoads direct loads
// of the whole wave.  bnc (walls on y): 1 for row 0, whose v_y = +1 group
// would come from beyond the wall and bounces back instead (it is read from
// the row itself, runs -v_i), 2 for row ny - 1 (the v_y = -1 group
// likewise), 0 otherwise.
// (The gather columns come as a plain pointer: taken as a reference to
// Gather<S, NC>, the second instantiation of the kernel for the same S and
// NC failed to compile.)
template <class S, int NC>
__device__ __forceinline__ void stage_row(const char* fin, const Params<float>& p, const uint32_t* gat_col,
                                          const uint32_t* gat_adj, int bnc, int lane, int r, char* dst_in) {
  using B = BlockLayout<S, 9>;
  // The LDS destination is passed through an empty asm statement: the
  // compiler's own tracking of direct loads into LDS would otherwise add a
  // vmcnt(0) before reads of the slot, which also waits for the stores the
  // explicit waits leave in flight.
  __attribute__((address_space(3))) char* dst = (__attribute__((address_space(3))) char*)dst_in;
  asm volatile("" : "+s"(dst));
  using G = Staged<S, NC>;
  const uint32_t stride = uint32_t(p.nbx) * uint32_t(NC * B::kComp);
  // row parts of the source rows of the groups v_y = 0, +1 (row above), -1
  const uint32_t ry0 = uint32_t(r) * stride;
  const uint32_t ry[3] = {ry0, bnc == 1 ? ry0 : uint32_t(wrap_add(r, -1, p.ny)) * stride,
                          bnc == 2 ? ry0 : uint32_t(wrap_add(r, 1, p.ny)) * stride};
#pragma unroll
  for (int j = 0; j < G::kLoads; ++j) {
    // the chunk's source row (known at compile time except for a load that
    // straddles two groups)
    const int ch = j * 64 + lane;
    const int g = ch < G::chunks(0) ? 0 : (ch < G::chunks(0) + G::chunks(1) ? 1 : 2);
    const uint32_t rp = g == 0 ? ry[0] : (g == 1 ? ry[1] : ry[2]);
    const uint32_t hop = bnc != 0 && g == bnc ? gat_adj[j] : 0u;
    __builtin_amdgcn_global_load_lds(fin + (rp + gat_col[j] + hop), dst + 1024u * uint32_t(j), 16, 0, 0);
  }
}

__device__ __forceinline__ _Float16 lds_half(const char* a) { return *reinterpret_cast<const _Float16*>(a); }
__device__ __forceinline__ float lds_f32(const char* a) { return *reinterpret_cast<const float*>(a); }

template <class S>
__device__ __forceinline__ float lds_raw(const char* a, int i) {
  if (i == 0) return float(*reinterpret_cast<const typename S::Rest*>(a));
  return float(*reinterpret_cast<const typename S::Move*>(a));
}

// W: the box has walls on y (p.walls == 2), a separate instantiation, so the
// periodic sweep carries none of their logic.
template <class S, int NC, bool W>
__global__ void __launch_bounds__(256) k_sweep_d2q9(const void* fin_v, void* fout,
                                                    Params<float> p, int strips, int seg_rows, int ntiles,
                                                    int tiles_per_xcd) {
  using L = Lattice<2>;
  using T = float;
  using B = BlockLayout<S, 9>;
  using G = Staged<S, NC>;
  __shared__ T s_rho[kRhoRing][NC][kRW];
  __shared__ T s_h[kHRing][NC][kHW];
  __shared__ __attribute__((aligned(16))) char s_stage[4][G::kBytes];
  const char* fin = static_cast<const char*>(fin_v);

  const int b = blockIdx.x;
  const int t = (b % kXcds) * tiles_per_xcd + b / kXcds;
  if (t >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform over the wave
  const int x0 = (t % strips) * kW;
  const int ya = (t / strips) * seg_rows;
  const int yb = min(ya + seg_rows, p.ny);
  const int rounds = (yb - ya + 3) / 4;
  const int ny = p.ny;

  // ring slots of virtual row r (r >= ya - 8 always)
  auto rslot = [&](int r) { return (r - ya + 8 * kRhoRing) & (kRhoRing - 1); };
  auto hslot = [&](int r) { return (r - ya + 8 * kHRing) & (kHRing - 1); };
  // walls on y: the row whose values the stencils use for virtual row v (the
  // layer next to a wall stands for the layer beyond it), and the bounce of
  // a staged virtual row v (stage_row's bnc)
  auto mrow = [&](int v) __attribute__((always_inline)) {
    if constexpr (W) return v < 0 ? -1 - v : (v >= ny ? 2 * ny - 1 - v : v);
    return v;
  };
  auto bnc_of = [&](int v) __attribute__((always_inline)) {
    if constexpr (W) return v == 0 ? 1 : (v == ny - 1 ? 2 : 0);
    return 0;
  };

  // Scale of the component of a halo lane (lane % NC), picked by selects
  // and kept in a register: an indexed read of the parameters would be a
  // vector memory load inside the rounds, whose wait would also wait for
  // the stores in flight.
  float halo_scale = 0.f;
  if constexpr (S::kShift) {
    const int c = lane % NC;
    halo_scale = p.sh.scale[0];
#pragma unroll
    for (int q = 1; q < NC; ++q) halo_scale = c == q ? p.sh.scale[q] : halo_scale;
    asm volatile("" : "+v"(halo_scale));
  }

  // Take a staged row into registers: decoded populations, in direction
  // order, and the running sum of each component (take_slot, take_shifted).
  // bnc: the staged row's bounce (stage_row); a bounced group's runs are the
  // row's own runs -v_i, read at the lane's own column.
  auto take = [&](const char* st, T (&f)[NC][9], T (&ledger)[NC], int bnc) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T led = T(0);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        // column lane - v_x of the padded segment (-1 and 64 in the halo parts)
        const bool own = bnc != 0 && bnc == G::group_of(i);
        const int col = own ? lane : lane - L::cx(i);
        const char* at = st + G::run0(c, i) + col * int(i == 0 ? B::kRest : B::kMove);
        if constexpr (S::kShift) {
          const _Float16 h = lds_half(st + G::ref0(c, L::cy(i)) + col * 2);
          take_shifted<2>(i, i == 0 ? _Float16(0) : lds_half(at), i == 0 ? lds_f32(at) : 0.f, h, p.sh.scale[c],
                          p.sh.one, led, f[c][i]);
        } else {
          take_slot<S, 2>(i, lds_raw<S>(at, i), led, f[c][i]);
        }
      }
      ledger[c] = led;
    }
  };
  // densities of virtual row r from taken populations
  auto put_rho = [&](int r, const T (&f)[NC][9], const T (&ledger)[NC]) __attribute__((always_inline)) {
    const int sr = rslot(r);
#pragma unroll
    for (int c = 0; c < NC; ++c) s_rho[sr][c][lane + 2] = site_density<S>(ledger[c], p.sh.scale[c]);
  };
  // densities of the four halo columns (-2, -1, 64, 65) of virtual row r:
  // lane hc * NC + c sums its nine pulled values in direction order (the
  // lane's component varies over the lanes: its scale is the one picked
  // once per lane above)
  auto put_rho_halo = [&](int r, const char* st, int bnc) __attribute__((always_inline)) {
    if (lane < 4 * NC) {
      const int hc = lane / NC, c = lane % NC;
      const int hcol = hc < 2 ? hc - 2 : kW + hc - 2;
      T v[9], led = T(0);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const bool own = bnc != 0 && bnc == G::group_of(i);
        const int col = own ? hcol : hcol - L::cx(i);  // -3 .. 66, inside the padded segment
        const char* at = st + G::run0(c, i) + col * int(i == 0 ? B::kRest : B::kMove);
        if constexpr (S::kShift) {
          const _Float16 h = lds_half(st + G::ref0(c, L::cy(i)) + col * 2);
          take_shifted<2>(i, i == 0 ? _Float16(0) : lds_half(at), i == 0 ? lds_f32(at) : 0.f, h, halo_scale,
                          p.sh.one, led, v[i]);
        } else {
          take_slot<S, 2>(i, lds_raw<S>(at, i), led, v[i]);
        }
      }
      s_rho[rslot(r)][c][hc < 2 ? hc : kW + hc] = site_density<S>(led, halo_scale);
    }
  };

  // potential h of virtual row r at h position q (column x0 - 1 + q)
  auto put_h = [&](int r, int q) __attribute__((always_inline)) {
    const int s0 = rslot(mrow(r - 1)), s1 = rslot(r), s2 = rslot(mrow(r + 1));
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
    site_potential<T, NC, true>(p, rr, lap, mu, hh);  // instantiated for N itself
    const int sh = hslot(r);
#pragma unroll
    for (int c = 0; c < NC; ++c) s_h[sh][c][q] = hh[c];
  };
  // h of rows r0 .. r0+3: each wave its own row's 64 interior columns, wave 0
  // the eight edge columns (q = 0 and 65) of all four rows
  auto put_h4 = [&](int r0) __attribute__((always_inline)) {
    put_h(r0 + w, lane + 1);
    if (w == 0 && lane < 8) put_h(r0 + (lane >> 1), (lane & 1) ? kHW - 1 : 0);
  };

  // collision of row rc from the populations and sums taken one round
  // earlier, in place (shifted codec: Fc then holds the stored deviations,
  // Lc the stored rest value, Hc the new references)
  auto collide_row = [&](int rc, T (&Fc)[NC][9], T (&Lc)[NC], float (&Hc)[NC]) __attribute__((always_inline)) {
    const int sr = rslot(rc);
    T rs[NC], jx[NC], jy[NC];
    T rt = T(0), ux = T(0), uy = T(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T ax = T(0), ay = T(0);
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        if (L::cx(i)) ax = L::cx(i) > 0 ? ax + Fc[c][i] : ax - Fc[c][i];
        if (L::cy(i)) ay = L::cy(i) > 0 ? ay + Fc[c][i] : ay - Fc[c][i];
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
    const int h0 = hslot(mrow(rc - 1)), h1 = hslot(rc), h2 = hslot(mrow(rc + 1));
    const int r0 = rslot(mrow(rc - 1)), r2 = rslot(mrow(rc + 1));
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
      T f[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = Fc[c][i];
      collide<2, T>(f, rs[c], ux, uy, T(0), Ax, Ay, Az, jx[c] * inv_rs, jy[c] * inv_rs, T(0), p.inv_tau);
      if constexpr (S::kShift) {
        // the site's new reference, the FP16 deviations of the moving
        // populations, and the rest of the ledger
        const float h = float(new_ref(Lc[c]));
        _Float16 d[9];
#pragma unroll
        for (int i = 1; i < 9; ++i) d[i] = encode_move<2>(i, f[i], p.sh.inv_scale[c], h);
        Lc[c] = ledger_rest<9>(Lc[c], h, d, p.sh.minus_one);
#pragma unroll
        for (int i = 1; i < 9; ++i) Fc[c][i] = float(d[i]);
        Hc[c] = h;
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) Fc[c][i] = f[i];
      }
    }
  };
  // non-temporal stores of a collided row: exactly Staged::kStores store
  // instructions (one per run, and one per reference run; runs are 256 or
  // 128 bytes apart, so none merge), which the wait at the start of the
  // next round counts on
  auto store_row = [&](int rc, const T (&Fc)[NC][9], const T (&Lc)[NC], const float (&Hc)[NC]) __attribute__((always_inline)) {
    const uint32_t orow = (uint32_t(rc) * uint32_t(p.nbx) + uint32_t(x0 >> 6)) * uint32_t(NC * B::kComp);
    const uint32_t own_rest = orow + B::in_run(0, lane), own_move = orow + B::in_run(1, lane);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      char* const outc = static_cast<char*>(fout) + B::run(c, 0);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const uint32_t off = (i == 0 ? own_rest : own_move) + (B::run(c, i) - B::run(c, 0));
        if constexpr (S::kShift) {
          if (i == 0)
            __builtin_nontemporal_store(Lc[c], reinterpret_cast<float*>(outc + off));
          else
            __builtin_nontemporal_store(_Float16(Fc[c][i]), reinterpret_cast<_Float16*>(outc + off));
        } else {
          __builtin_nontemporal_store(Fc[c][i], reinterpret_cast<T*>(outc + off));
        }
      }
      if constexpr (S::kShift)
        __builtin_nontemporal_store(_Float16(Hc[c]), reinterpret_cast<_Float16*>(static_cast<char*>(fout) + orow +
                                                                                 B::ref(c) + B::in_ref(lane)));
    }
  };

  T F0[NC][9], L0[NC], F1[NC][9], L1[NC];
  float H0[NC];
  char* const stage = s_stage[w];
  const Gather<S, NC> gat = make_gather<S, NC>(p, lane, x0);

  // ---- prologue --------------------------------------------------------
  // rho of rows ya-2, ya-1 (waves 2, 3) and ya .. ya+3 (all waves); h of rows
  // ya-1 .. ya+2; populations of row ya + w in F0; row ya + 4 + w staged.
  if (w >= 2) {
    stage_row<S, NC>(fin, p, gat.col, gat.adj, bnc_of(ya - 4 + w), lane, wrap_mod(ya - 4 + w, ny), stage);
    wait_vm<0>();
    take(stage, F1, L1, bnc_of(ya - 4 + w));
    put_rho(ya - 4 + w, F1, L1);
    put_rho_halo(ya - 4 + w, stage, bnc_of(ya - 4 + w));
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the slot is read before it is staged again
  }
  stage_row<S, NC>(fin, p, gat.col, gat.adj, bnc_of(ya + w), lane, wrap_mod(ya + w, ny), stage);
  wait_vm<0>();
  take(stage, F0, L0, bnc_of(ya + w));
  put_rho(ya + w, F0, L0);
  put_rho_halo(ya + w, stage, bnc_of(ya + w));
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  stage_row<S, NC>(fin, p, gat.col, gat.adj, bnc_of(ya + 4 + w), lane, wrap_mod(ya + 4 + w, ny), stage);
  lds_barrier();
  put_h4(ya - 1);
  lds_barrier();

  // ---- rounds ------------------------------------------------------------
  // Round k takes row ra = rc + 4 (staged in the round before) into F1 and
  // collides row rc = ya + 4k + w from F0, then moves F1 into F0.  Vector
  // memory operations retire in issue order, and a round that collided
  // issued its kStores stores after its staging loads, so the next round
  // waits until at most kStores operations remain in flight: the staged row
  // has landed, the stores complete during that round.  In a full round
  // every wave collides and stores unconditionally; rounds 1 .. full - 1 are
  // entered only from full rounds, so the compiler's own wait before the
  // first read of the staged row counts the same stores.
  auto round = [&](int k, bool full, bool prev_stored) __attribute__((always_inline)) {
    const int rc = ya + 4 * k + w;
    const int ra = rc + 4;
    if (prev_stored)
      wait_vm<G::kStores>();
    else
      wait_vm<0>();
    take(stage, F1, L1, bnc_of(ra));
    put_rho(ra, F1, L1);
    put_rho_halo(ra, stage, bnc_of(ra));
    if (k + 1 < rounds) {
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the slot is read before it is staged again
      // shifted FP16: the wave issues its staging loads at raised priority,
      // ahead of the other waves' arithmetic (2.5% faster at 2048^2; the same
      // for FP32 is 4% slower)
      if constexpr (S::kShift) __builtin_amdgcn_s_setprio(1);
      stage_row<S, NC>(fin, p, gat.col, gat.adj, bnc_of(ra + 4), lane, wrap_mod(ra + 4, ny), stage);
      if constexpr (S::kShift) __builtin_amdgcn_s_setprio(0);
    }
    lds_barrier();
    put_h4(ya + 4 * k + 3);
    lds_barrier();
    if (full || rc < yb) {
      collide_row(rc, F0, L0, H0);
      store_row(rc, F0, L0, H0);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int i = 0; i < 9; ++i) F0[c][i] = F1[c][i];
      L0[c] = L1[c];
    }
  };
  const int full = (yb - ya) / 4;  // rounds in which all four waves collide
  if (full > 0) {
    round(0, true, false);
    for (int k = 1; k < full; ++k) round(k, true, true);
    if (full < rounds) round(full, false, true);
  } else {
    round(0, false, false);  // a segment of fewer than four rows
  }
}

}  // namespace sweep

// Rows per segment: about one workgroup per resident slot (as many per CU as
// registers and LDS allow), rounded up to whole rounds of four rows, so the
// grid runs in one wave of workgroups and the rows re-read at segment ends
// stay a small fraction of it.
static int sweep_rows(int nx, int ny, int slots) {
  const int strips = nx / 64;
  const int segs = (slots + strips - 1) / strips;
  int rows = (ny + segs - 1) / segs;
  rows = (rows + 3) / 4 * 4;
  return rows < 4 ? 4 : rows;
}

// Resident workgroups of the sweep kernel on the current device.
template <class S, int NC, bool W>
static int sweep_slots_of() {
  static const int slots = [] {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep::k_sweep_d2q9<S, NC, W>, 256, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    return per_cu * cus;
  }();
  return slots;
}

// Resident workgroups of the instantiation that run p launches (walls on y
// or not).
template <class S, int NC>
static int sweep_slots(const Params<float>& p) {
  return (p.walls & 2) ? sweep_slots_of<S, NC, true>() : sweep_slots_of<S, NC, false>();
}

template <class S, int NC>
static void launch_rows(const Ctx& c, const void* fin, void* fout, int rows) {
  const Params<float>& p = c.params<float>();
  const int strips = p.nx / 64;
  const int ntiles = strips * ((p.ny + rows - 1) / rows);
  const int per_xcd = (ntiles + sweep::kXcds - 1) / sweep::kXcds;
  // walls: on y only (the context takes the sweep for no other)
  if (p.walls & 2)
    sweep::k_sweep_d2q9<S, NC, true><<<per_xcd * sweep::kXcds, 256, 0, c.stream>>>(fin, fout, p, strips, rows, ntiles,
                                                                                   per_xcd);
  else
    sweep::k_sweep_d2q9<S, NC, false><<<per_xcd * sweep::kXcds, 256, 0, c.stream>>>(fin, fout, p, strips, rows,
                                                                                    ntiles, per_xcd);
}

template <class S, int NC>
static void launch_sweep(const Ctx& c, const void* fin, void* fout) {
  const Params<float>& p = c.params<float>();
  launch_rows<S, NC>(c, fin, fout, c.sweep_rows > 0 ? c.sweep_rows : sweep_rows(p.nx, p.ny, sweep_slots<S, NC>(p)));
}

// Segment lengths worth timing for this run, the one-wave default first.
// Large grids only: there the time also depends on how the segments fall on
// the workgroup slots and the L2s (neighbouring short segments share their
// halo rows in L2), irregularly enough to be measured rather than predicted.
template <class S, int NC>
static int candidates(const Ctx& c, int* cand) {
  const Params<float>& p = c.params<float>();
  if (static_cast<long long>(p.nx) * p.ny < (1LL << 20)) return 0;
  const int top = (p.ny + 3) / 4 * 4;
  int nc = 0;
  auto add = [&](int r) {
    r = r > top ? top : r;
    for (int i = 0; i < nc; ++i)
      if (cand[i] == r) return;
    cand[nc++] = r;
  };
  add(sweep_rows(p.nx, p.ny, sweep_slots<S, NC>(p)));
  for (int r : {16, 24, 32, 48, 64, 96, 128}) add(r);
  return nc;
}

template <class S>
static int candidates_for_n(const Ctx& c, int* cand) {
  switch (c.prm.n_comp) {
    case 1: return candidates<S, 1>(c, cand);
    case 2: return candidates<S, 2>(c, cand);
    case 3: return candidates<S, 3>(c, cand);
    case 4: return candidates<S, 4>(c, cand);
    default: return 0;
  }
}

int sweep_candidates(const Ctx& c, int* cand) {
  if (c.prm.storage == StoreF32::kId) return candidates_for_n<StoreF32>(c, cand);
  if (c.prm.storage == StoreF16S::kId) return candidates_for_n<StoreF16S>(c, cand);
  return 0;
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

// FP32 and shifted FP16 only: FP64 would halve the rows that fit in LDS and
// registers.
FusedStepFn sweep_step_for(int storage, int n_comp) {
  if (storage == StoreF32::kId) return sweep_for_n<StoreF32>(n_comp);
  if (storage == StoreF16S::kId) return sweep_for_n<StoreF16S>(n_comp);
  return nullptr;
}

}  // namespace lbm
