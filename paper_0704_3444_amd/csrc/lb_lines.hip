// Groups of one-dimensional runs stepped together (lb_lines_* of the C ABI).
//
// The phase-equilibrium experiments of Sec. IV are D1Q3 runs on short
// periodic lines, many of them (one per interaction strength, relaxation
// time or starting composition), each over tens of thousands of steps.  A
// whole line fits in the registers of one wavefront: lane l owns the P
// consecutive sites x = P l ... P l + P - 1 of a line of nx = 64 P sites.
// A launch reads each run's populations once, takes all the requested steps
// with the populations and every per-site quantity in registers, and writes
// the populations once.  Within a step the neighbours x - 1 and x + 1 of a
// site are in the same lane except at the ends of a lane's run of sites;
// those come from the neighbouring lane by a rotation of the wavefront by
// one lane, which also closes the periodic line (lane 63's right neighbour
// is lane 0).  No LDS and no barrier is used.
//
// Each step performs the operations of the split path in their order
// (k_density, k_potential, k_collide of k_split.hip) through the same
// per-site functions of physics.hpp, so a run stepped in a group and the
// same run stepped by lb_step hold the same populations bit for bit.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lb.h"
#include "lbm_internal.hpp"
#include "storage.hpp"

namespace lbm {
namespace lines {

constexpr int kMaxSitesPerLane = 4;  // nx <= 256
constexpr int kMaxLineComp = 4;

// What the kernel needs of one run (device memory, written at group
// creation).
template <typename T>
struct Run {
  Params<T> p;
  void* f[2];  // the context's two population copies
  int* flag;   // the context's sticky health flag
  int pad[2];
};

// Value of v held by lane (lane + d) mod 64, d = -1 or +1: a DPP rotation
// of the whole wavefront by one lane (wave_ror:1 brings lane l - 1 to lane
// l, wave_rol:1 lane l + 1), 32 bits at a time.
__device__ __forceinline__ int rotate32(int v, int d) {
  return d < 0 ? __builtin_amdgcn_update_dpp(0, v, 0x13C, 0xF, 0xF, false)   // wave_ror:1
               : __builtin_amdgcn_update_dpp(0, v, 0x134, 0xF, 0xF, false);  // wave_rol:1
}
__device__ __forceinline__ float rotate(float v, int d) {
  return __int_as_float(rotate32(__float_as_int(v), d));
}
__device__ __forceinline__ double rotate(double v, int d) {
  const long long b = __double_as_longlong(v);
  const int lo = rotate32(int(b & 0xffffffffll), d), hi = rotate32(int(b >> 32), d);
  return __longlong_as_double((long long)(unsigned(lo)) | ((long long)hi << 32));
}

template <typename T>
__device__ __forceinline__ bool unhealthy(T r) {
  return !(r > T(0)) || !(r < (sizeof(T) == 8 ? T(1e300) : T(3e38f)));
}

// nsteps steps of every run of the group: workgroup r (one wavefront) holds
// run r.  fin = f[par], fout = f[par ^ 1] for every run.
template <class S, int NC, int P>
__global__ void __launch_bounds__(64) k_lines(const Run<typename S::T>* __restrict__ runs, int par,
                                              long long nsteps) {
  using T = typename S::T;
  using L = Lattice<1>;
  constexpr int Q = 3;
  static_assert(!S::kShift, "plain codecs only");
  const Run<T>& run = runs[blockIdx.x];
  const Params<T> p = run.p;
  const char* fin = static_cast<const char*>(run.f[par]);
  char* fout = static_cast<char*>(run.f[par ^ 1]);
  const int lane = threadIdx.x;
  const int nx = 64 * P;

  // populations pulled into the lane's sites: f_i(x) is slot (i, x - v_i)
  T f[NC][P][Q];
#pragma unroll
  for (int k = 0; k < NC; ++k)
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int src = wrap_add(lane * P + j, -L::cx(i), nx);
        f[k][j][i] = load_slot<S>(fin, pop_byte<S, Q>(NC, p.nbx, k, i, src, 0), i);
      }

  bool bad = false;
  for (long long step = 0; step < nsteps; ++step) {
    // densities (k_density)
    T rho[NC][P];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int j = 0; j < P; ++j) {
        T acc = T(0);  // the split path's density: the sum in direction order
#pragma unroll
        for (int i = 0; i < Q; ++i) acc += f[k][j][i];
        rho[k][j] = acc;
        bad |= unhealthy(rho[k][j]);
      }
    // neighbour densities rho(x - 1), rho(x + 1)
    T rl[NC][P], rr[NC][P];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T from_left = rotate(rho[k][P - 1], -1);
      const T from_right = rotate(rho[k][0], +1);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        rl[k][j] = j > 0 ? rho[k][j - 1] : from_left;
        rr[k][j] = j < P - 1 ? rho[k][j + 1] : from_right;
      }
    }
    // potentials (k_potential); i = 1 is v = +1, i = 2 is v = -1
    T h[NC][P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      T r[NC], lap[NC], mu[NC], hs[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        r[k] = rho[k][j];
        lap[k] = lattice_laplacian<1, T>([&](int i) { return i == 1 ? rr[k][j] : rl[k][j]; }, r[k]);
      }
      site_potential<T, NC, true>(p, r, lap, mu, hs);  // a group has one N, NC
#pragma unroll
      for (int k = 0; k < NC; ++k) h[k][j] = hs[k];
    }
    T hl[NC][P], hr[NC][P];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T from_left = rotate(h[k][P - 1], -1);
      const T from_right = rotate(h[k][0], +1);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        hl[k][j] = j > 0 ? h[k][j - 1] : from_left;
        hr[k][j] = j < P - 1 ? h[k][j + 1] : from_right;
      }
    }
    // force, equilibrium, forcing term, BGK (k_collide)
#pragma unroll
    for (int j = 0; j < P; ++j) {
      T jx[NC];
      T rt = T(0), ux = T(0);
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        T ax = T(0);
        ax += T(L::cx(1)) * f[k][j][1];
        ax += T(L::cx(2)) * f[k][j][2];
        jx[k] = ax;
        ux += ax;
        rt += rho[k][j];
      }
      const T inv_rt = rcp_(rt);
      ux *= inv_rt;
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const T rs = rho[k][j];
        T Ax, Ay, Az;
        lattice_force<1, T>([&](int i) { return i == 1 ? hr[k][j] : hl[k][j]; },
                            [&](int i) { return i == 1 ? rr[k][j] : rl[k][j]; }, rs, p, Ax, Ay, Az);
        const T inv_rs = rcp_(rs);
        collide<1, T>(f[k][j], rs, ux, T(0), T(0), Ax, Ay, Az, jx[k] * inv_rs, T(0), T(0), p.inv_tau);
      }
    }
    // streaming: f_1 (v = +1) moves one site right, f_2 one site left
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T in1 = rotate(f[k][P - 1][1], -1);
      const T in2 = rotate(f[k][0][2], +1);
#pragma unroll
      for (int j = P - 1; j > 0; --j) f[k][j][1] = f[k][j - 1][1];
      f[k][0][1] = in1;
#pragma unroll
      for (int j = 0; j < P - 1; ++j) f[k][j][2] = f[k][j + 1][2];
      f[k][P - 1][2] = in2;
    }
  }

  // back to pull storage: the value pulled into x along v_i is slot (i, x - v_i)
#pragma unroll
  for (int k = 0; k < NC; ++k)
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int dst = wrap_add(lane * P + j, -L::cx(i), nx);
        *reinterpret_cast<T*>(fout + pop_byte<S, Q>(NC, p.nbx, k, i, dst, 0)) = f[k][j][i];
      }
  if (__ballot(bad) != 0ull && lane == 0) *run.flag = 1;
}

template <class S, int NC, int P>
void launch(const void* runs, int nruns, int par, long long nsteps, hipStream_t s) {
  k_lines<S, NC, P><<<nruns, 64, 0, s>>>(static_cast<const Run<typename S::T>*>(runs), par, nsteps);
}

using LaunchFn = void (*)(const void*, int, int, long long, hipStream_t);

template <class S, int NC>
LaunchFn pick_p(int P) {
  switch (P) {
    case 1: return launch<S, NC, 1>;
    case 2: return launch<S, NC, 2>;
    case 3: return launch<S, NC, 3>;
    case 4: return launch<S, NC, 4>;
    default: return nullptr;
  }
}

template <class S>
LaunchFn pick_n(int n, int P) {
  switch (n) {
    case 1: return pick_p<S, 1>(P);
    case 2: return pick_p<S, 2>(P);
    case 3: return pick_p<S, 3>(P);
    case 4: return pick_p<S, 4>(P);
    default: return nullptr;
  }
}

LaunchFn pick(int storage, int n, int P) {
  if (storage == LB_F64) return pick_n<StoreF64>(n, P);
  if (storage == LB_F32) return pick_n<StoreF32>(n, P);
  return nullptr;
}

}  // namespace lines
}  // namespace lbm

struct lb_lines {
  std::vector<lb_ctx*> ctxs;
  void* runs = nullptr;  // device array of Run<T>
  lbm::lines::LaunchFn launch = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;  // every member context's current copy
};

namespace {

template <typename T>
void fill_runs(const std::vector<lb_ctx*>& ctxs, std::vector<char>* bytes) {
  using R = lbm::lines::Run<T>;
  bytes->assign(ctxs.size() * sizeof(R), 0);
  for (size_t r = 0; r < ctxs.size(); ++r) {
    R run;
    std::memset(&run, 0, sizeof(run));
    const lbm::Ctx& c = ctxs[r]->c;
    run.p = c.params<T>();
    run.f[0] = c.f[0];
    run.f[1] = c.f[1];
    run.flag = c.health_flag;
    std::memcpy(bytes->data() + r * sizeof(R), &run, sizeof(R));
  }
}

}  // namespace

extern "C" {

int lb_lines_create(lb_ctx* const* ctxs, int32_t n, lb_lines** out) {
  using lbm::fail_with;
  if (!out) return fail_with(LB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctxs || n < 1) return fail_with(LB_EINVAL, "need at least one context");
  if (n > (1 << 20)) return fail_with(LB_EINVAL, "too many contexts");
  if (!ctxs[0]) return fail_with(LB_EINVAL, "context 0 is NULL");
  const lbm::Ctx& c0 = ctxs[0]->c;
  for (int r = 0; r < n; ++r) {
    const lb_ctx* h = ctxs[r];
    if (!h) return fail_with(LB_EINVAL, ("context " + std::to_string(r) + " is NULL").c_str());
    const lbm::Ctx& c = h->c;
    const std::string at = " (context " + std::to_string(r) + ")";
    if (c.prm.lattice != LB_D1Q3) return fail_with(LB_ENOTSUP, ("groups hold D1Q3 runs only" + at).c_str());
    if (c.prm.storage != LB_F64 && c.prm.storage != LB_F32)
      return fail_with(LB_ENOTSUP, ("groups hold LB_F64 or LB_F32 runs only" + at).c_str());
    if (c.prm.nx % 64 != 0 || c.prm.nx / 64 > lbm::lines::kMaxSitesPerLane)
      return fail_with(LB_ENOTSUP, ("nx must be 64, 128, 192 or 256" + at).c_str());
    if (c.prm.n_comp > lbm::lines::kMaxLineComp) return fail_with(LB_ENOTSUP, ("N must be <= 4" + at).c_str());
    if (c.prm.walls != 0) return fail_with(LB_ENOTSUP, ("groups hold periodic lines only" + at).c_str());
    if (c.prm.n_comp != c0.prm.n_comp || c.prm.storage != c0.prm.storage || c.prm.nx != c0.prm.nx)
      return fail_with(LB_EINVAL, ("every run of a group needs the same N, storage and nx" + at).c_str());
    if (c.stream != c0.stream) return fail_with(LB_EINVAL, ("every run of a group needs the same stream" + at).c_str());
    if (c.cur != c0.cur) return fail_with(LB_EINVAL, ("every run of a group must be on the same one of its two population copies" + at).c_str());
    for (int q = 0; q < r; ++q)
      if (ctxs[q] == h) return fail_with(LB_EINVAL, ("a context appears twice" + at).c_str());
  }
  lbm::lines::LaunchFn fn = lbm::lines::pick(c0.prm.storage, c0.prm.n_comp, int(c0.prm.nx / 64));
  if (!fn) return fail_with(LB_ENOTSUP, "no kernel for this storage / N / nx");
  lb_lines* g = new (std::nothrow) lb_lines;
  if (!g) return fail_with(LB_ENOMEM, "host allocation failed");
  g->ctxs.assign(ctxs, ctxs + n);
  g->launch = fn;
  g->stream = c0.stream;
  g->cur = c0.cur;
  std::vector<char> bytes;
  if (c0.prm.storage == LB_F64)
    fill_runs<double>(g->ctxs, &bytes);
  else
    fill_runs<float>(g->ctxs, &bytes);
  hipError_t e = hipMalloc(&g->runs, bytes.size());
  if (e != hipSuccess) {
    delete g;
    return fail_with(LB_ENOMEM, (std::string("hipMalloc of the run table: ") + hipGetErrorString(e)).c_str());
  }
  e = hipMemcpyAsync(g->runs, bytes.data(), bytes.size(), hipMemcpyHostToDevice, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) {
    (void)hipFree(g->runs);
    delete g;
    return fail_with(LB_EDEVICE, (std::string("upload of the run table: ") + hipGetErrorString(e)).c_str());
  }
  *out = g;
  return LB_OK;
}

int lb_lines_step(lb_lines* g, int64_t nsteps) {
  using lbm::fail_with;
  if (!g) return fail_with(LB_EINVAL, "group is NULL");
  if (nsteps < 0) return fail_with(LB_EINVAL, "nsteps must be >= 0");
  for (size_t r = 0; r < g->ctxs.size(); ++r)
    if (g->ctxs[r]->c.cur != g->cur)
      return fail_with(LB_EINVAL, ("context " + std::to_string(r) + " has changed copies outside the group").c_str());
  if (nsteps == 0) return LB_OK;
  g->launch(g->runs, int(g->ctxs.size()), g->cur, static_cast<long long>(nsteps), g->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_with(LB_EDEVICE, (std::string("k_lines launch: ") + hipGetErrorString(e)).c_str());
  g->cur ^= 1;
  for (lb_ctx* h : g->ctxs) {
    h->c.cur = g->cur;
    h->c.t += nsteps;
  }
  return LB_OK;
}

void lb_lines_free(lb_lines* g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  (void)hipFree(g->runs);
  delete g;
}

}  // extern "C"
