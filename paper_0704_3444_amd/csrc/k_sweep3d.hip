// Plane-sweep D3Q19 step: one launch per time step, every population read
// from memory once and written once.
//
// A workgroup owns a pencil of 64 x-sites (one 64-site block of the
// population layout) by kTY rows and a segment of z-planes, which it sweeps
// upwards.  It has one wave per (row, component) unit of the pencil, 4 N
// waves.  The collision of plane z needs the potentials h of planes z - 1 ..
// z + 1 and the densities of planes z - 1 .. z + 1; h of plane z + 1 needs
// the Laplacian of the densities, so densities run two planes ahead of the
// collision.  One iteration, for the collision of plane zc:
//   1. every wave issues the loads of its unit in plane zc + 3 and writes
//      the first moments of its unit in plane zc to LDS;
//   2. (barrier) chemical potentials and h of plane zc + 1 on the rows and
//      columns the force stencil reaches, into an LDS ring;
//   3. (barrier) the loads of the halo-column pieces of plane zc + 4, a plane
//      ahead of the rest (they are scattered over many cache lines and land
//      last); force, equilibrium, forcing term and collision of plane zc from
//      the registers; non-temporal stores in place (the next step's pull
//      streams them);
//   4. the 19 populations of plane zc + 3 land in registers; the wave writes
//      their density to an LDS ring and keeps them: each wave holds three
//      planes of its unit (zc + 1 .. zc + 3 after the step), so each
//      population is loaded once.  It also sums the densities of one unit of
//      the two halo rows above and below the pencil and of 8 sites of the
//      halo columns (two on either side), which the neighbouring pencils load
//      as their own (mostly L2 hits).
// Each site's arithmetic is the split path's (the same physics.hpp functions
// with the same operands in the same order), so the two agree bit for bit.
// Workgroups are banded per XCD so that neighbouring pencils share an L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbm_internal.hpp"
#include "physics.hpp"
#include "storage.hpp"

namespace lbm {
namespace sweep3 {

constexpr int kXcds = 8;
constexpr int kW = 64;          // pencil width = block width = wave size
constexpr int kTY = 4;          // rows per pencil
constexpr int kRP = 5;          // density planes in LDS (zc - 2 .. zc + 2 live)
constexpr int kHP = 3;          // h planes in LDS (zc - 1 .. zc + 1 live)
constexpr int kJP = 2;          // first-moment planes in LDS (zc and zc + 1 live)
constexpr int kRR = kTY + 4;    // density rows: y0 - 2 .. y0 + kTY + 1
constexpr int kRC = kW + 4;     // density columns: x0 - 2 .. x0 + 65
constexpr int kHR = kTY + 2;    // h rows: y0 - 1 .. y0 + kTY
constexpr int kHC = kW + 2;     // h columns: x0 - 1 .. x0 + 64

// Workgroup barrier that publishes this wave's LDS writes without waiting
// for its global loads and stores in flight (no wave reads global memory
// that another wave of the step writes).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ int wrap_mod(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}

// Ring slot of virtual plane z (z >= za - 2).
template <int R>
__device__ __forceinline__ int slot(int z, int za) {
  return (z - za + 2 * R) % R;
}

// Pieces of the halo columns, per density row of a wave (2 rows): for every
// direction i the 16 bytes at the end of run i of the block left of the
// pencil ("left", columns x0 - 4 .. x0 - 1 of a 4-byte run) and at the start
// of run i of the block right of it ("right", x0 + 64 .. x0 + 67), and, for
// the 5 directions with v_x = -1 and the 5 with v_x = +1, the first and the
// last 16 bytes of run i of the pencil's own block ("own start", column x0,
// pulled into x0 - 1; "own end", x0 + 63, pulled into x0 + 64).  The pieces
// of a row sit in kSlotsPerRow 16-byte slots, arranged so that every halo
// column finds the slot value it pulls from run i at one fixed offset from
// its own base: left piece of run i at slot left_slot(i), followed by the own
// start of i where v_x(i) = -1; right piece at left_slot(i) + kRightShift,
// preceded by the own end of i where v_x(i) = +1.  Column x0 + s (s = -2, -1)
// then reads run i at byte 16 left_slot(i) - 4 v_x(i) + 4 (s + 4), column
// x0 + 64 + s (s = 0, 1) at 16 left_slot(i) - 4 v_x(i) + 16 kRightShift + 4 s:
// one LDS read with an immediate offset per direction.  Slots 0 .. 14 hold
// the x-pairs k = 0 .. 4 (left of x_plus(k), left of x_plus(k) + 1, own start
// of x_plus(k) + 1), 15 .. 23 the left pieces of the 9 directions with
// v_x = 0, 24 .. 38 (own end of x_plus(k), right of x_plus(k), right of
// x_plus(k) + 1), 39 is unused, 40 .. 48 the right pieces of v_x = 0.
constexpr int kSlotsPerRow = 49;
constexpr int kRightShift = 25;
constexpr int kPieces = 2 * kSlotsPerRow;

// the k-th direction with v_x = +1 (its opposite, v_x = -1, is the next one)
__host__ __device__ constexpr int x_plus(int k) { return k == 0 ? 1 : 2 * k + 5; }
// the n-th direction with v_x = 0
__host__ __device__ constexpr int x_zero(int n) { return n == 0 ? 0 : (n < 5 ? n + 2 : n + 10); }

__host__ __device__ constexpr int left_slot(int i) {
  for (int k = 0; k < 5; ++k) {
    if (i == x_plus(k)) return 3 * k;
    if (i == x_plus(k) + 1) return 3 * k + 1;
  }
  for (int n = 0; n < 9; ++n)
    if (i == x_zero(n)) return 15 + n;
  return -1;
}

constexpr bool piece_slots_consistent() {
  // every direction has a slot; v_x = -1 leaves the next slot to its own
  // start, v_x = +1 the slot before its right piece to its own end
  for (int i = 0; i < 19; ++i) {
    const int s = left_slot(i);
    if (s < 0 || s + kRightShift >= kSlotsPerRow) return false;
    for (int j = 0; j < 19; ++j) {
      if (j != i && left_slot(j) == s) return false;
      if (Lattice<3>::cx(i) == -1 && left_slot(j) == s + 1) return false;
      if (Lattice<3>::cx(i) == 1 && left_slot(j) == s - 1) return false;
    }
  }
  return kRightShift >= 15 + 9;  // the right pieces after all left slots
}
static_assert(piece_slots_consistent(), "halo-column piece slots");

enum PieceKind { kLeftEnd, kOwnStart, kOwnEnd, kRightStart };

// Direction and kind of the piece in slot idx of a row (slot 39, unused,
// loads the left piece of the rest run again).
__device__ __forceinline__ void piece_of(int idx, int& i, int& kind) {
  if (idx < 15) {
    const int k = idx / 3, m = idx - 3 * (idx / 3);
    i = x_plus(k) + (m == 0 ? 0 : 1);
    kind = m == 2 ? kOwnStart : kLeftEnd;
  } else if (idx < 24) {
    i = x_zero(idx - 15);
    kind = kLeftEnd;
  } else if (idx < 39) {
    const int k = (idx - 24) / 3, m = (idx - 24) - 3 * ((idx - 24) / 3);
    i = x_plus(k) + (m == 2 ? 1 : 0);
    kind = m == 0 ? kOwnEnd : kRightStart;
  } else if (idx == 39) {
    i = 0;
    kind = kLeftEnd;
  } else {
    i = x_zero(idx - 40);
    kind = kRightStart;
  }
}

// Per-wave staging, filled by direct global-to-LDS loads: the halo-row unit
// of one plane (19 pulled values per lane) and the halo-column pieces of two
// planes (by parity of the plane).
struct Stage {
  uint32_t unit[19][kW];
  uint32_t piece[2][kPieces][4];
};

template <class S, int NC>
struct Smem {
  float rho[kRP][NC][kRR][kRC];
  float h[kHP][NC][kHR][kHC];
  float j[kJP][3][NC][kTY][kW];
  Stage st[kTY * NC];
};

// Byte offset of population i of component c at site (x, y, z), 32-bit
// (the fused paths are taken only for copies below 4 GiB).
template <class S, int NC>
__device__ __forceinline__ uint32_t pop_off(const Params<float>& p, int c, int i, int x, int y, int z) {
  using B = BlockLayout<S, 19>;
  const uint32_t row = uint32_t(y) + uint32_t(p.ny) * uint32_t(z);
  return (row * uint32_t(p.nbx) + uint32_t(x >> 6)) * uint32_t(NC * B::kComp) + B::run(c, i) + B::in_run(i, x);
}

// Per-lane part of a population's byte offset: the block of column x
// (taken from the lane's source column) and the position in the run, for
// the rest run (4-byte slots) and for moving runs.  The row part is the
// same for the whole wave.
struct LanePart {
  uint32_t rest;     // column x, rest run
  uint32_t move[3];  // moving runs, source column x - d for d = -1, 0, +1 (index d + 1)
};

template <class S, int NC>
__device__ __forceinline__ LanePart lane_part(const Params<float>& p, int x) {
  using B = BlockLayout<S, 19>;
  constexpr uint32_t comp = NC * B::kComp;
  LanePart lp;
  lp.rest = uint32_t(x >> 6) * comp + B::in_run(0, x);
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    const int sx = wrap_add(x, -d, p.nx);
    lp.move[d + 1] = uint32_t(sx >> 6) * comp + B::in_run(1, sx);
  }
  return lp;
}

// Raw buffer resource over a population copy of `bytes` bytes (gfx9
// family: 4th descriptor word 0x00020000, stride 0, byte offsets).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// One FP32 slot through the buffer resource (row and run part of the offset
// in an SGPR, the lane's column part in a VGPR).
__device__ __forceinline__ float load_slot32(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}

// 16 bytes per lane from byte offset voff of the buffer into LDS at dst +
// 16 lane (a direct load: no registers hold the data in flight).  Kept out
// of the kernel body: there the 16-byte form of the builtin made the host
// pass drop the kernel's instantiation without a diagnostic.
__device__ __forceinline__ void load_lds16(__amdgpu_buffer_rsrc_t rs, __attribute__((address_space(3))) char* dst,
                                           uint32_t voff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dst, 16, voff, 0u, 0, 0);
}

// s_waitcnt vmcnt(N), the other counters untouched, as a compiler memory
// barrier.
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// W: the box has walls on z (p.walls == 4), a separate instantiation, so the
// periodic sweep carries none of their logic.
template <class S, int NC, bool W>
__global__ void __launch_bounds__(64 * kTY * NC) k_sweep_d3q19(const void* fin_v, void* fout_v, Params<float> p,
                                                               int strips, int ytiles, int seg, int ntiles,
                                                               int tiles_per_xcd) {
  using L = Lattice<3>;
  using T = float;
  using B = BlockLayout<S, 19>;
  static_assert(!S::kShift && B::kRest == 4 && B::kMove == 4, "FP32 slots only");
  __shared__ Smem<S, NC> sm;
  const uint32_t copy_bytes = uint32_t(p.ny) * uint32_t(p.nz) * uint32_t(p.nbx) * uint32_t(NC * B::kComp);
  const __amdgpu_buffer_rsrc_t fin = buffer_of(fin_v, copy_bytes);
  const __amdgpu_buffer_rsrc_t fout = buffer_of(fout_v, copy_bytes);

  const int b = blockIdx.x;
  const int t = (b % kXcds) * tiles_per_xcd + b / kXcds;
  if (t >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = w / NC;  // own row 0 .. kTY - 1
  const int c = w % NC;  // component of all this wave's units
  // tile order: strip fastest, then y-tile, then z-segment
  const int x0 = (t % strips) * kW;
  const int y0 = ((t / strips) % ytiles) * kTY;
  const int za = (t / (strips * ytiles)) * seg;
  const int zb = min(za + seg, p.nz);
  const int nplanes = zb - za;

  // coordinates of this wave's own unit, halo-row unit and halo-column sites
  const int x = x0 + lane;
  const int y_own = y0 + r;
  const int hrow = r < 2 ? r : kTY + r;  // density row of the halo unit: 0, 1, kTY + 2, kTY + 3
  const int y_halo = wrap_mod(y0 - 2 + hrow, p.ny);
  // halo columns: lanes 0 .. 7 take columns x0 - 2, x0 - 1, x0 + 64, x0 + 65
  // (lane % 4) of the density row 2 r + lane / 4
  const int hcol = lane & 3, hpass = (lane >> 2) & 1;
  const int xcol_lds = hcol < 2 ? hcol : kW + hcol;                        // 0, 1, 66, 67
  const int hbase = hpass * kSlotsPerRow * 16 + (hcol < 2 ? 4 * (hcol + 2) : 16 * kRightShift + 4 * (hcol - 2));
  const LanePart lp_own = lane_part<S, NC>(p, x);
  const uint32_t stride = uint32_t(p.nbx) * uint32_t(NC * B::kComp);  // bytes per row of blocks
  // the piece each lane loads in the two 16-byte loads of the halo columns:
  // density row 2 r + prow[j], source row offsets (pdy, pdz), and the part of
  // its byte offset that does not depend on the row
  int prow[2], pdy[2], pdz[2];
  uint32_t pcol[2], padj[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int q = j * kW + lane;
    const int qq = q < kPieces ? q : 0;
    const int idx = qq % kSlotsPerRow;
    int i, kind;
    piece_of(idx, i, kind);
    const int bx = kind == kLeftEnd ? wrap_mod(x0 - 1, p.nx) >> 6
                 : (kind == kRightStart ? wrap_mod(x0 + kW, p.nx) >> 6 : x0 >> 6);
    const bool at_end = kind == kLeftEnd || kind == kOwnEnd;
    const uint32_t esz = i == 0 ? B::kRest : B::kMove;
    prow[j] = qq / kSlotsPerRow;
    pdy[j] = L::cy(i);
    pdz[j] = L::cz(i);
    pcol[j] = uint32_t(bx) * uint32_t(NC * B::kComp) + B::run(c, i) + (at_end ? kW * esz - 16u : 0u);
    padj[j] = B::run(c, L::opp(i)) - B::run(c, i);  // to the same piece of the opposite run
  }

  // Walls on z: whether direction i, pulled into virtual plane z, would come
  // from beyond a wall (v_z = +1 into plane 0, -1 into plane nz - 1); it
  // then bounces back: the site's own population -v_i, read at the site
  // itself.  mz: the plane whose densities and potentials the stencils use
  // for virtual plane v (the plane next to a wall stands for the one beyond).
  const int nz = p.nz;
  auto bounced = [&](int z, int dz) __attribute__((always_inline)) {
    if constexpr (W) return dz > 0 ? z == 0 : (dz < 0 ? z == nz - 1 : false);
    return false;
  };
  auto mz = [&](int v) __attribute__((always_inline)) {
    if constexpr (W) return v < 0 ? -1 - v : (v >= nz ? 2 * nz - 1 - v : v);
    return v;
  };
  // The loads of the own and halo-row units of a plane next to a wall take a
  // branch of their own, so that the other planes' loads carry no selects.
  auto at_wall = [&](int z) __attribute__((always_inline)) { return z == 0 || z == nz - 1; };

  // The staging slot's LDS address is passed through an empty asm
  // statement: the compiler's own tracking of direct loads into LDS would
  // otherwise add a vmcnt(0) before reads of the slot, which would also wait
  // for the stores in flight; the explicit waits below order them instead.
  __attribute__((address_space(3))) char* stg = (__attribute__((address_space(3))) char*)(&sm.st[w]);
  asm volatile("" : "+s"(stg));

  // byte offset of source row y - dy of plane z - dz
  auto rowb = [&](int y, int z, int dy, int dz) __attribute__((always_inline)) {
    return (uint32_t(wrap_add(y, -dy, p.ny)) + uint32_t(p.ny) * uint32_t(wrap_add(z, -dz, p.nz))) * stride;
  };
  // column part of a staged load's offset, aligned down to 4 bytes
  auto col_off = [&](const LanePart& lp, int i) __attribute__((always_inline)) -> uint32_t {
    return (i == 0 ? lp.rest : lp.move[L::cx(i) + 1]) & ~3u;
  };

  // The own unit's populations: X holds the raw slots of the plane in
  // flight; D0, D1, D2 the decoded populations of planes zc, zc + 1, zc + 2
  // (L0, L1, L2 their ledgers, shifted codec).  Each iteration decodes X
  // into D2, loads the next plane into X and moves D1 -> D0, D2 -> D1, so
  // that every set keeps one place in registers.
  float X[19], D0[19], D1[19], D2[19], L0 = 0.f, L1 = 0.f, L2 = 0.f;

  // The halo-column pieces of virtual plane z into this wave's staging (by
  // parity of z).
  // (Its two loads select their offsets per lane instead: with the loads in
  // both branches, the compiler merged them under the lane condition and
  // passed their common LDS destination through a VGPR.)
  auto issue_pieces = [&](int z) __attribute__((always_inline)) {
    const int zw = wrap_mod(z, p.nz);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j * kW + lane < kPieces) {
        const int yr = wrap_mod(y0 - 2 + 2 * r + prow[j], p.ny);
        uint32_t off = rowb(yr, zw, pdy[j], pdz[j]) + pcol[j];
        if constexpr (W) off = bounced(z, pdz[j]) ? rowb(yr, zw, 0, 0) + pcol[j] + padj[j] : off;
        load_lds16(fin, stg + (19 * kW * 4 + (z & 1) * kPieces * 16 + j * kW * 16), off);
      }
    }
  };

  // Issue the loads of virtual plane z: the halo-row unit into this wave's
  // staging, the own unit into register set Pn, then (in the prologue) the
  // pieces of plane z + 1; in the iterations those follow later (see there).
  // consume(z) waits until at most 21 vector memory operations are in
  // flight: in the prologue the own unit's 19 loads and the two of the next
  // pieces follow the halo-row unit's loads, in the iterations the two of
  // the next pieces and the collision's 19 stores follow the own unit's.
  // Either way the halo-row unit has landed, and so have the pieces of
  // plane z, issued before both.
  auto issue = [&](int z, float (&Pn)[19], bool next_pieces) __attribute__((always_inline)) {
    const int zw = wrap_mod(z, p.nz);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // this wave's reads of the staging are done
    // walls: the loads of both units, for a plane next to a wall (WP) or not
    auto body = [&](auto wall) __attribute__((always_inline)) {
      constexpr bool WP = decltype(wall)::value;
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const bool bo = WP && bounced(z, L::cz(i));
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            fin, stg + i * (kW * 4), 4, bo ? lp_own.move[1] : col_off(lp_own, i),
            bo ? rowb(y_halo, zw, 0, 0) + B::run(c, L::opp(i)) : rowb(y_halo, zw, L::cy(i), L::cz(i)) + B::run(c, i),
            0, 0);
      }
      asm volatile("" ::: "memory");  // the own unit's loads after the halo-row unit's
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const bool bo = WP && bounced(z, L::cz(i));
        const uint32_t so =
            bo ? rowb(y_own, zw, 0, 0) + B::run(c, L::opp(i)) : rowb(y_own, zw, L::cy(i), L::cz(i)) + B::run(c, i);
        const uint32_t vo = bo ? lp_own.move[1] : (i == 0 ? lp_own.rest : lp_own.move[L::cx(i) + 1]);
        Pn[i] = load_slot32(fin, vo, so);
      }
    };
    if constexpr (W) {
      if (at_wall(z))
        body(std::true_type{});
      else
        body(std::false_type{});
    } else {
      // periodic box: the same loads written out (through the generic body
      // the compiler scheduled the periodic kernel differently)
#pragma unroll
      for (int i = 0; i < 19; ++i)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(fin, stg + i * (kW * 4), 4, col_off(lp_own, i),
                                                 rowb(y_halo, zw, L::cy(i), L::cz(i)) + B::run(c, i), 0, 0);
      asm volatile("" ::: "memory");  // the own unit's loads after the halo-row unit's
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const uint32_t so = rowb(y_own, zw, L::cy(i), L::cz(i)) + B::run(c, i);
        const uint32_t vo = i == 0 ? lp_own.rest : lp_own.move[L::cx(i) + 1];
        Pn[i] = load_slot32(fin, vo, so);
      }
    }
    if (next_pieces) {
      asm volatile("" ::: "memory");  // the next pieces after the own unit's loads
      issue_pieces(z + 1);
    }
  };

  // First moments of this wave's unit in virtual plane z from its populations
  // f, into the LDS ring.
  auto moments = [&](int z, const float (&f)[19]) __attribute__((always_inline)) {
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      if (L::cx(i)) ax += T(L::cx(i)) * f[i];
      if (L::cy(i)) ay += T(L::cy(i)) * f[i];
      if (L::cz(i)) az += T(L::cz(i)) * f[i];
    }
    const int js = slot<kJP>(z, za);
    sm.j[js][0][c][r][lane] = ax;
    sm.j[js][1][c][r][lane] = ay;
    sm.j[js][2][c][r][lane] = az;
  };

  // Step 4 for virtual plane z, loads issued by issue(z, Xr): densities of
  // the own unit (decoded from Xr into Dd, with its ledger Ld), of the
  // halo-row unit and of the halo-column sites.
  auto consume = [&](int z, const float (&Xr)[19], float (&Dd)[19], float& Ld) __attribute__((always_inline)) {
    const int rs = slot<kRP>(z, za);
    {
      float led = 0.f;
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const float v = Xr[i];
        led = i == 0 ? v : led + v;
        Dd[i] = v;
      }
      sm.rho[rs][c][r + 2][lane + 2] = led;
      Ld = led;
    }
    wait_vm<21>();  // the halo-row unit and the pieces of plane z have landed
    const uint32_t* su = reinterpret_cast<const uint32_t*>(&sm.st[w].unit[0][0]);
    {
      float led = 0.f;
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const float v = __builtin_bit_cast(float, su[i * kW + lane]);
        led = i == 0 ? v : led + v;
      }
      sm.rho[rs][c][hrow][lane + 2] = led;
    }
    if (lane < 8) {
      const char* base = reinterpret_cast<const char*>(&sm.st[w].piece[z & 1][0][0]) + hbase;
      // WP: plane next to a wall (its reads then take a branch of their own,
      // with immediate offsets like the others)
      auto body = [&](auto wall) __attribute__((always_inline)) {
        float led = 0.f;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
          // a bounced run was loaded into the same pieces from the site's
          // own row and plane: its value sits at the column itself
          const int sh = decltype(wall)::value && bounced(z, L::cz(i)) ? 0 : -4 * L::cx(i);
          const float v = *reinterpret_cast<const float*>(base + 16 * left_slot(i) + sh);
          led = i == 0 ? v : led + v;
        }
        sm.rho[rs][c][2 * r + hpass][xcol_lds] = led;
      };
      if constexpr (W) {
        if (at_wall(z))
          body(std::true_type{});
        else
          body(std::false_type{});
      } else {
        float led = 0.f;  // the periodic box's reads written out (see issue)
#pragma unroll
        for (int i = 0; i < 19; ++i) {
          const float v = *reinterpret_cast<const float*>(base + 16 * left_slot(i) - 4 * L::cx(i));
          led = i == 0 ? v : led + v;
        }
        sm.rho[rs][c][2 * r + hpass][xcol_lds] = led;
      }
    }
  };

  // Step 2 for virtual plane z: potentials h on the kHR x kHC sites around
  // the pencil, all components at once.
  auto potentials = [&](int z) __attribute__((always_inline)) {
    const int s0 = slot<kRP>(mz(z - 1), za), s1 = slot<kRP>(z, za), s2 = slot<kRP>(mz(z + 1), za);
    const int hs = slot<kHP>(z, za);
    for (int q = threadIdx.x; q < kHR * kHC; q += 64 * kTY * NC) {
      const int hr = q / kHC, hc = q - hr * kHC;
      const int pr = hr + 1, pc = hc + 1;  // density row and column of the site
      T rr[NC], lap[NC], mu[NC], hh[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        rr[k] = sm.rho[s1][k][pr][pc];
        lap[k] = lattice_laplacian<3, T>(
            [&](int i) {
              const int sz = L::cz(i) > 0 ? s2 : (L::cz(i) < 0 ? s0 : s1);
              return sm.rho[sz][k][pr + L::cy(i)][pc + L::cx(i)];
            },
            rr[k]);
      }
      site_potential<T, NC, true>(p, rr, lap, mu, hh);  // instantiated for N itself
#pragma unroll
      for (int k = 0; k < NC; ++k) sm.h[hs][k][hr][hc] = hh[k];
    }
  };

  // Step 3 for virtual plane z from register set f: collision of this
  // wave's unit and its 19 stores.
  auto collide_store = [&](int z, float (&f)[19], float led) __attribute__((always_inline)) {
    const int zw = wrap_mod(z, p.nz);
    const int s0 = slot<kRP>(mz(z - 1), za), s1 = slot<kRP>(z, za), s2 = slot<kRP>(mz(z + 1), za);
    const int h0 = slot<kHP>(mz(z - 1), za), h1 = slot<kHP>(z, za), h2 = slot<kHP>(mz(z + 1), za);
    const int js = slot<kJP>(z, za);
    T rt = T(0), ux = T(0), uy = T(0), uz = T(0);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      ux += sm.j[js][0][k][r][lane];
      uy += sm.j[js][1][k][r][lane];
      uz += sm.j[js][2][k][r][lane];
      rt += sm.rho[s1][k][r + 2][lane + 2];
    }
    const T inv_rt = rcp_(rt);
    ux *= inv_rt;
    uy *= inv_rt;
    uz *= inv_rt;
    const T rs = sm.rho[s1][c][r + 2][lane + 2];
    // the force of lattice_force (physics.hpp), term by term, with the
    // potential's and the density's neighbour reads in two groups
    T hx, hy, hz;
    lattice_wsum<3, T>(
        [&](int i) {
          const int hp = L::cz(i) > 0 ? h2 : (L::cz(i) < 0 ? h0 : h1);
          return sm.h[hp][c][r + 1 + L::cy(i)][lane + 1 + L::cx(i)];
        },
        hx, hy, hz);
    asm volatile("" ::: "memory");
    T qx = T(0), qy = T(0), qz = T(0);
    if (!p.log_form)
      lattice_wsum<3, T>(
          [&](int i) {
            const int sz = L::cz(i) > 0 ? s2 : (L::cz(i) < 0 ? s0 : s1);
            return sm.rho[sz][c][r + 2 + L::cy(i)][lane + 2 + L::cx(i)];
          },
          qx, qy, qz);
    const T Ax = -p.cforce * fma_(rs, T(3) * hx, -qx);
    const T Ay = -p.cforce * fma_(rs, T(3) * hy, -qy);
    const T Az = -p.cforce * fma_(rs, T(3) * hz, -qz);
    const T inv_rs = rcp_(rs);
    const T jx = sm.j[js][0][c][r][lane], jy = sm.j[js][1][c][r][lane], jz = sm.j[js][2][c][r][lane];
    collide<3, T>(f, rs, ux, uy, uz, Ax, Ay, Az, jx * inv_rs, jy * inv_rs, jz * inv_rs, p.inv_tau);
    // non-temporal buffer stores (policy bit nt): the row and run part of
    // each slot's offset in an SGPR, the lane's column part in a VGPR.  The
    // wave issues them at raised priority, ahead of the other waves'
    // arithmetic, so that the stores of a plane leave the CU together.
    const uint32_t row = rowb(y_own, zw, 0, 0);
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int i = 0; i < 19; ++i)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, f[i]), fout, lp_own.rest,
                                            row + B::run(c, i), 2);
    __builtin_amdgcn_s_setprio(0);
  };

  // ---- prologue: densities of planes za - 2 .. za + 2 (the last three kept
  // in D0, D1 and D2), potentials of planes za - 1 and za
  issue_pieces(za - 2);
  issue(za - 2, X, true);
  consume(za - 2, X, D2, L2);
  issue(za - 1, X, true);
  consume(za - 1, X, D2, L2);
  issue(za, X, true);
  consume(za, X, D0, L0);
  issue(za + 1, X, true);
  consume(za + 1, X, D1, L1);
  issue(za + 2, X, true);
  consume(za + 2, X, D2, L2);
  lds_barrier();
  potentials(za - 1);
  potentials(za);

  // ---- iterations: plane zc + 3 is loaded into X first, so that its loads
  // are in flight during the potentials of plane zc + 1 and the collision of
  // plane zc (D0), and consumed into D2 after that collision's stores, so
  // that the waits for X leave exactly those stores in flight (X is never in
  // flight at the top of the loop).  The pieces of plane zc + 4 are issued
  // between the potentials and the collision: half an iteration before the
  // neighbouring pencils load the blocks they come from (at the top of the
  // next iteration), so those lines are mostly still in L2 then, and an
  // iteration and a half before they are read.
  for (int k = 0; k < nplanes; ++k) {
    const int zc = za + k;
    issue(zc + 3, X, false);
    moments(zc, D0);
    lds_barrier();
    potentials(zc + 1);
    lds_barrier();
    issue_pieces(zc + 4);
    collide_store(zc, D0, L0);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      D0[i] = D1[i];
      D1[i] = D2[i];
    }
    L0 = L1;
    L1 = L2;
    consume(zc + 3, X, D2, L2);
  }
}

}  // namespace sweep3

// Resident workgroups of the D3Q19 sweep on the current device.
template <class S, int NC, bool W>
static int sweep3_slots() {
  static const int slots = [] {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep3::k_sweep_d3q19<S, NC, W>, 64 * sweep3::kTY * NC,
                                                     0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    return per_cu * cus;
  }();
  return slots;
}

// Planes per z-segment: about one workgroup per resident slot, so that the
// grid runs in one wave of workgroups; each segment re-reads 4 planes of
// densities at its start.
template <class S, int NC>
static void launch_sweep3(const Ctx& c, const void* fin, void* fout) {
  const Params<float>& p = c.params<float>();
  const int strips = p.nx / sweep3::kW;
  const int ytiles = p.ny / sweep3::kTY;
  const int pencils = strips * ytiles;
  const int slots = (p.walls & 4) ? sweep3_slots<S, NC, true>() : sweep3_slots<S, NC, false>();
  const int segs = std::max(1, std::min(p.nz, (slots + pencils - 1) / pencils));
  const int seg = (p.nz + segs - 1) / segs;
  const int ntiles = pencils * ((p.nz + seg - 1) / seg);
  const int per_xcd = (ntiles + sweep3::kXcds - 1) / sweep3::kXcds;
  // walls: on z only (the context takes the sweep for no other)
  if (p.walls & 4)
    sweep3::k_sweep_d3q19<S, NC, true><<<per_xcd * sweep3::kXcds, 64 * sweep3::kTY * NC, 0, c.stream>>>(
        fin, fout, p, strips, ytiles, seg, ntiles, per_xcd);
  else
    sweep3::k_sweep_d3q19<S, NC, false><<<per_xcd * sweep3::kXcds, 64 * sweep3::kTY * NC, 0, c.stream>>>(
        fin, fout, p, strips, ytiles, seg, ntiles, per_xcd);
}

template <class S>
static FusedStepFn sweep3_for_n(int n_comp) {
  switch (n_comp) {
    case 1: return launch_sweep3<S, 1>;
    case 2: return launch_sweep3<S, 2>;
    case 3: return launch_sweep3<S, 3>;
    default: return nullptr;  // N = 4 would need 16 waves of at most 128 VGPRs: it spills
  }
}

// D3Q19 plane sweep: FP32, N <= 3; the caller checks nx % 64 == 0, ny % 4 ==
// 0, walls on z at most and a copy below 4 GiB.  The shifted FP16 codec takes the split
// path: its decode needs the references of the 19 source sites of every
// unit, halo rows and columns included, which the pencil's registers and
// LDS (full at N = 3) do not hold.
FusedStepFn sweep3d_step_for(int storage, int n_comp) {
  if (storage == StoreF32::kId) return sweep3_for_n<StoreF32>(n_comp);
  return nullptr;
}

}  // namespace lbm
