// C ABI of the library (declared in include/lb.h): parameter validation,
// workspace layout, the step loop, observables and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "lb.h"
#include "lbm_internal.hpp"

using lbm::Ctx;

// Device scratch of lb_moments_noalloc: the FP64 field buffers of the
// observables (rho, mu, h, U, P), for callers that cannot allocate.  Each
// device holds its own copy of the array; host code uses only the address
// hipGetSymbolAddress gives for the current device, never the array's name.
static __device__ __align__(256) unsigned char scratch[LB_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on device dev (the current device), looked up once
// per device; nullptr with the HIP error on failure.
void* scratch_on(int dev, hipError_t* err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int lattice_dims(int lattice, int* Q, int* D) {
  switch (lattice) {
    case LB_D1Q3: *Q = 3; *D = 1; return 0;
    case LB_D2Q9: *Q = 9; *D = 2; return 0;
    case LB_D3Q19: *Q = 19; *D = 3; return 0;
    default: return -1;
  }
}

int validate(const lb_params* p, std::string* why) {
  auto bad = [&](const std::string& m) { *why = m; return LB_EINVAL; };
  if (!p) return bad("params is NULL");
  int Q, D;
  if (lattice_dims(p->lattice, &Q, &D)) return bad("unknown lattice");
  if (p->n_comp < 1 || p->n_comp > LB_MAX_COMP) return bad("n_comp must be in 1..8");
  if (p->storage != LB_F64 && p->storage != LB_F32 && p->storage != LB_F16S) return bad("unknown storage");
  if (p->force_form != LB_FORCE_LOG && p->force_form != LB_FORCE_EXPANDED) return bad("unknown force_form");
  if (p->path < LB_PATH_AUTO || p->path > LB_PATH_SWEEP) return bad("unknown path");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return bad("box sides must be >= 1");
  if (p->nx > (1 << 30) || p->ny > (1 << 30) || p->nz > (1 << 30)) return bad("box side too large");
  if (p->lattice == LB_D1Q3 && (p->ny != 1 || p->nz != 1)) return bad("D1Q3 needs ny = nz = 1");
  if (p->lattice == LB_D2Q9 && p->nz != 1) return bad("D2Q9 needs nz = 1");
  const double S = double(p->nx) * double(p->ny) * double(p->nz);
  if (S * p->n_comp * Q > 4.0e12) return bad("lattice too large");
  const int N = p->n_comp;
  for (int k = 0; k < N; ++k) {
    if (!std::isfinite(p->tau[k]) || !(p->tau[k] > 0.5)) return bad("tau must be > 1/2");
    if (p->tau[k] != p->tau[0])
      return bad("all tau^sigma must be equal (one total-fluid LB equation needs one tau)");
    if (!std::isfinite(p->m[k]) || !(p->m[k] > 0.0)) return bad("m^sigma must be > 0");
  }
  if (!std::isfinite(p->theta) || !(p->theta > 0.0)) return bad("theta must be > 0");
  if (!std::isfinite(p->kappa) || !(p->kappa >= 0.0)) return bad("kappa must be >= 0");
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      const double v = p->chi[a * LB_MAX_COMP + b];
      if (!std::isfinite(v)) return bad("chi must be finite");
      if (v != p->chi[b * LB_MAX_COMP + a]) return bad("chi must be symmetric");
      if (a == b && v != 0.0) return bad("chi^{sigma sigma} must be 0");
    }
  if (p->check_every < 0) return bad("check_every must be >= 0");
  if (p->walls & ~7) return bad("walls: only bits 0 (x), 1 (y) and 2 (z)");
  {
    int D2 = 0, Q2 = 0;
    lattice_dims(p->lattice, &Q2, &D2);
    if (p->walls >> D2) return bad("walls: an axis beyond the lattice's dimension");
    const int64_t side[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a)
      if (((p->walls >> a) & 1) && side[a] < 2) return bad("walls: a closed axis needs at least 2 layers");
  }
  if (p->reserved != 0) return bad("reserved must be 0");
  return LB_OK;
}

struct Layout {
  size_t f, rho, h, diag_partial, diag_out, flag, total;
  int diag_blocks;
};

// Bytes of one population copy: rows * (64-site blocks per row) * N * the
// bytes of one component's 64-site block (the x extent is padded to a
// multiple of 64; padded slots are never used).  A component's block holds
// 64 rest values and 64 (Q - 1) moving values: FP64 8 + 8, FP32 4 + 4,
// shifted FP16 4 (the FP32 ledger) + 2.
size_t population_bytes(const lb_params* p) {
  int Q, D;
  lattice_dims(p->lattice, &Q, &D);
  const size_t nbx = (size_t(p->nx) + 63) / 64;
  const size_t rest = p->storage == LB_F64 ? 8 : 4;
  const size_t move = p->storage == LB_F64 ? 8 : (p->storage == LB_F32 ? 4 : 2);
  const size_t ref = p->storage == LB_F16S ? 2 : 0;  // the shifted codec's reference run
  return size_t(p->ny) * size_t(p->nz) * nbx * size_t(p->n_comp) * 64 * (rest + ref + (Q - 1) * move);
}

// Bytes of the working precision (FP64 for LB_F64, FP32 otherwise).
size_t work_bytes(const lb_params* p) { return p->storage == LB_F64 ? 8 : 4; }

Layout layout_of(const lb_params* p) {
  int Q, D;
  lattice_dims(p->lattice, &Q, &D);
  const size_t S = size_t(p->nx) * size_t(p->ny) * size_t(p->nz);
  const size_t rb = work_bytes(p);
  Layout L;
  const size_t fbytes = align_up(population_bytes(p));
  const size_t rbytes = align_up(size_t(p->n_comp) * S * rb);
  const size_t blocks = (S + 255) / 256;
  L.diag_blocks = int(blocks < 1024 ? blocks : 1024);
  const int K = LB_MAX_COMP + D + 1;
  L.f = 0;
  L.rho = 2 * fbytes;
  L.h = L.rho + rbytes;
  L.diag_partial = L.h + rbytes;
  L.diag_out = L.diag_partial + align_up(size_t(L.diag_blocks) * K * sizeof(double));
  L.flag = L.diag_out + align_up(K * sizeof(double));
  L.total = L.flag + kAlign;
  return L;
}

template <typename T>
void fill_params(const lb_params* p, lbm::Params<T>* q) {
  std::memset(q, 0, sizeof(*q));
  q->n = p->n_comp;
  q->log_form = p->force_form == LB_FORCE_LOG ? 1 : 0;
  q->nx = int(p->nx);
  q->ny = int(p->ny);
  q->nz = int(p->nz);
  q->S = (long long)p->nx * p->ny * p->nz;
  q->nbx = int((p->nx + 63) / 64);
  int Q, D;
  lattice_dims(p->lattice, &Q, &D);
  q->nq = p->n_comp * Q;
  q->walls = p->walls;
  q->inv_tau = T(1.0 / p->tau[0]);
  q->cforce = T(1.0 - 0.5 / p->tau[0]);
  q->theta = T(p->theta);
  q->kappa = T(p->kappa);
  for (int k = 0; k < lbm::kMaxComp; ++k) q->inv_m[k] = T(k < p->n_comp ? 1.0 / p->m[k] : 1.0);
  for (int a = 0; a < lbm::kMaxComp; ++a)
    for (int b = 0; b < lbm::kMaxComp; ++b)
      q->chi[a * lbm::kMaxComp + b] =
          T(a < p->n_comp && b < p->n_comp ? p->chi[a * LB_MAX_COMP + b] : 0.0);
}

// Scale of the shifted FP16 storage from the initial densities: s^sigma =
// twice the smallest power of two >= max rho0^sigma (the pulled totals
// rho / s then stay below 1, where their FP32 sums are exact, until a density
// doubles that maximum).  Zero for the other codecs.
lbm::ShiftRef shift_ref_of(const lb_params* p, const double* rho0, size_t S) {
  lbm::ShiftRef r;
  std::memset(&r, 0, sizeof(r));
  if (p->storage != LB_F16S) return r;
  r.one = 1.0f;
  r.minus_one = -1.0f;
  for (int k = 0; k < p->n_comp; ++k) {
    double mx = 0.0;
    for (size_t i = 0; i < S; ++i) mx = std::max(mx, rho0[k * S + i]);
    int e = 0;
    std::frexp(mx, &e);  // mx = m 2^e with m in [0.5, 1)
    if (std::ldexp(1.0, e - 1) >= mx) e -= 1;  // mx itself a power of two
    e += 1;
    r.scale[k] = float(std::ldexp(1.0, e));
    r.inv_scale[k] = float(std::ldexp(1.0, -e));
  }
  return r;
}

// One time step of the context's path on its stream (no health check).
void step_once(Ctx& c) {
  void* fin = c.f[c.cur];
  void* fout = c.f[1 - c.cur];
  if (c.path != LB_PATH_SPLIT && c.fused)
    c.fused(c, fin, fout);
  else
    lbm::split_table(c.prm.lattice, c.prm.storage).step(c, fin, fout);
  c.cur = 1 - c.cur;
  c.t += 1;
}

// Segment length of the sweep (SweepTuner): trial steps on the context's
// state, timed with events on its stream; waits for the last event.  The
// caller restores the state afterwards.  On any HIP failure the one-wave
// default is kept.
void tune_sweep(Ctx& c) {
  using Tu = lbm::SweepTuner;
  int cand[Tu::kMax];
  const int nc = lbm::sweep_candidates(c, cand);
  c.sweep_rows = 0;
  if (nc <= 0) return;
  hipEvent_t ev[2 * Tu::kMax * Tu::passes] = {};
  const int nev = 2 * nc * Tu::passes;
  bool ok = true;
  for (int i = 0; ok && i < nev; ++i) ok = hipEventCreate(&ev[i]) == hipSuccess;
  if (ok) {
    for (int j = 0; j < Tu::warm; ++j) step_once(c);
    for (int q = 0; q < Tu::passes; ++q)
      for (int i = 0; i < nc; ++i) {
        const int e = 2 * (q * nc + i);
        c.sweep_rows = cand[i];
        step_once(c);
        (void)hipEventRecord(ev[e], c.stream);
        for (int j = 0; j < Tu::steps_per; ++j) step_once(c);
        (void)hipEventRecord(ev[e + 1], c.stream);
      }
    ok = hipEventSynchronize(ev[nev - 1]) == hipSuccess;
  }
  // the two lengths with the shortest trials
  int best = -1, second = -1;
  float best_ms = 0.f, second_ms = 0.f;
  for (int i = 0; ok && i < nc; ++i) {
    float ms_i = -1.f;
    for (int q = 0; q < Tu::passes; ++q) {
      const int e = 2 * (q * nc + i);
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[e], ev[e + 1]) != hipSuccess) continue;
      if (ms_i < 0.f || ms < ms_i) ms_i = ms;
    }
    if (ms_i < 0.f) continue;
    if (best < 0 || ms_i < best_ms) {
      second = best;
      second_ms = best_ms;
      best = i;
      best_ms = ms_i;
    } else if (second < 0 || ms_i < second_ms) {
      second = i;
      second_ms = ms_i;
    }
  }
  for (int i = 0; i < nev; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  // the two again, alternately, over longer runs: short trials separate
  // lengths a few percent apart, not the closest ones
  if (ok && second >= 0) {
    hipEvent_t rv[2 * 2 * Tu::rpasses] = {};
    const int nrv = 2 * 2 * Tu::rpasses;
    bool rok = true;
    for (int i = 0; rok && i < nrv; ++i) rok = hipEventCreate(&rv[i]) == hipSuccess;
    if (rok) {
      const int pick[2] = {best, second};
      for (int q = 0; q < Tu::rpasses; ++q)
        for (int j = 0; j < 2; ++j) {
          const int e = 2 * (2 * q + j);
          c.sweep_rows = cand[pick[j]];
          step_once(c);
          (void)hipEventRecord(rv[e], c.stream);
          for (int s = 0; s < Tu::rsteps; ++s) step_once(c);
          (void)hipEventRecord(rv[e + 1], c.stream);
        }
      rok = hipEventSynchronize(rv[nrv - 1]) == hipSuccess;
      float sum[2] = {0.f, 0.f};
      for (int q = 0; rok && q < Tu::rpasses; ++q)
        for (int j = 0; j < 2; ++j) {
          const int e = 2 * (2 * q + j);
          float ms = 0.f;
          rok = hipEventElapsedTime(&ms, rv[e], rv[e + 1]) == hipSuccess;
          sum[j] += ms;
        }
      if (rok && sum[1] < sum[0]) best = second;
    }
    for (int i = 0; i < nrv; ++i)
      if (rv[i]) (void)hipEventDestroy(rv[i]);
  }
  (void)hipGetLastError();
  c.sweep_rows = best >= 0 ? cand[best] : 0;
}

// Step the context's state n times on its stream.
int advance(Ctx& c, int64_t n) {
  const lbm::SplitTable& st = lbm::split_table(c.prm.lattice, c.prm.storage);
  for (int64_t k = 0; k < n; ++k) {
    step_once(c);
    if (c.prm.check_every > 0 && c.t % c.prm.check_every == 0) st.diag(c, c.f[c.cur]);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return LB_OK;
}

}  // namespace

extern "C" {

size_t lb_workspace_bytes(const lb_params* p) {
  std::string why;
  if (validate(p, &why) != LB_OK) {
    g_last_error = why;
    return 0;
  }
  return layout_of(p).total;
}

}  // extern "C"

namespace lbm {

// lb_init with an optional device staging buffer for rho0 (at least
// N * S doubles); without one, a buffer is allocated and freed here.
int init_impl(const lb_params* p, const double* rho0, void* workspace, size_t workspace_bytes, double* staging,
              bool tune, lb_ctx** out) {
  std::string why;
  if (!out) return fail(LB_EINVAL, "out is NULL");
  *out = nullptr;
  if (validate(p, &why) != LB_OK) return fail(LB_EINVAL, why);
  if (!rho0) return fail(LB_EINVAL, "rho0 is NULL");
  const size_t S = size_t(p->nx) * size_t(p->ny) * size_t(p->nz);
  for (size_t k = 0; k < size_t(p->n_comp) * S; ++k)
    if (!std::isfinite(rho0[k]) || !(rho0[k] > 0.0))
      return fail(LB_EINVAL, "rho0 must be finite and > 0 at every site (index " + std::to_string(k) + ")");
  const Layout L = layout_of(p);
  if (workspace) {
    if (workspace_bytes < L.total)
      return fail(LB_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
      return fail(LB_EINVAL, "workspace must be 256-byte aligned");
  }
  lb_ctx* h = new (std::nothrow) lb_ctx;
  if (!h) return fail(LB_ENOMEM, "host allocation failed");
  Ctx& c = h->c;
  c.prm = *p;
  lattice_dims(p->lattice, &c.Q, &c.D);
  c.S = (long long)S;
  c.real_bytes = work_bytes(p);
  c.pop_bytes = population_bytes(p);
  c.stream = static_cast<hipStream_t>(p->stream);
  if (hipGetDevice(&c.device) != hipSuccess) {
    delete h;
    return hip_fail(hipGetLastError(), "hipGetDevice");
  }
  {
    // the address of lb_moments_noalloc's scratch on this device, looked up
    // here once per device; a failure is reported by that call instead
    hipError_t se = hipSuccess;
    (void)scratch_on(c.device, &se);
  }
  if (workspace) {
    c.ws = workspace;
    c.ws_bytes = workspace_bytes;
  } else {
    hipError_t e = hipMalloc(&c.ws, L.total);
    if (e != hipSuccess) {
      delete h;
      return fail(LB_ENOMEM, std::string("hipMalloc of workspace: ") + hipGetErrorString(e));
    }
    c.owns_ws = true;
    c.ws_bytes = L.total;
  }
  char* base = static_cast<char*>(c.ws);
  const size_t fbytes = c.pop_bytes;
  c.f[0] = base + L.f;
  c.f[1] = base + L.f + align_up(fbytes);
  c.rho_scratch = base + L.rho;
  c.h_scratch = base + L.h;
  c.diag_partial = reinterpret_cast<double*>(base + L.diag_partial);
  c.diag_out = reinterpret_cast<double*>(base + L.diag_out);
  c.health_flag = reinterpret_cast<int*>(base + L.flag);
  c.diag_blocks = L.diag_blocks;
  fill_params(p, &c.pf);
  fill_params(p, &c.pd);
  c.pf.sh = c.pd.sh = shift_ref_of(p, rho0, S);

  // the fused kernels address one population copy with 32-bit byte offsets;
  // walls: the split path, the D2Q9 tile kernel, and the sweeps when they
  // close only the swept axis (y on D2Q9, z on D3Q19)
  const bool fits = fbytes < (size_t(1) << 32);
  lbm::FusedStepFn tile = fits && (p->walls == 0 || p->lattice == LB_D2Q9)
                              ? lbm::fused_step_for(p->lattice, p->storage, p->n_comp)
                              : nullptr;
  lbm::FusedStepFn sweep = fits && (p->walls & ~2) == 0 && p->lattice == LB_D2Q9 && p->nx % 64 == 0
                               ? lbm::sweep_step_for(p->storage, p->n_comp)
                               : nullptr;
  if (fits && (p->walls & ~4) == 0 && p->lattice == LB_D3Q19 && p->nx % 64 == 0 && p->ny % 4 == 0)
    sweep = lbm::sweep3d_step_for(p->storage, p->n_comp);
  switch (p->path) {
    case LB_PATH_AUTO:
      c.path = sweep ? LB_PATH_SWEEP : (tile ? LB_PATH_TILE : LB_PATH_SPLIT);
      break;
    case LB_PATH_TILE:
      c.path = LB_PATH_TILE;
      if (!tile) {
        lb_free(h);
        return fail(LB_ENOTSUP, "no tile kernel for this lattice / storage / N / size / walls");
      }
      break;
    case LB_PATH_SWEEP:
      c.path = LB_PATH_SWEEP;
      if (!sweep) {
        lb_free(h);
        return fail(LB_ENOTSUP, "the sweep kernels need D2Q9 (FP32 or shifted FP16, N <= 4) or D3Q19 (FP32, N <= 3, ny a multiple of 4), nx a multiple of 64; walls only on the swept axis, y on D2Q9 and z on D3Q19");
      }
      break;
    default:
      c.path = LB_PATH_SPLIT;
  }
  c.fused = c.path == LB_PATH_SWEEP ? sweep : (c.path == LB_PATH_TILE ? tile : nullptr);

  double* rho_dev = staging;
  hipError_t e = hipSuccess;
  if (!rho_dev) {
    e = hipMalloc(&rho_dev, size_t(p->n_comp) * S * sizeof(double));
    if (e != hipSuccess) {
      lb_free(h);
      return fail(LB_ENOMEM, std::string("hipMalloc of rho0 staging: ") + hipGetErrorString(e));
    }
  }
  e = hipMemcpyAsync(rho_dev, rho0, size_t(p->n_comp) * S * sizeof(double), hipMemcpyHostToDevice, c.stream);
  if (e == hipSuccess) e = hipMemsetAsync(c.health_flag, 0, sizeof(int), c.stream);
  // padded slots (x >= nx in the last block of a row) are never written by
  // the step; clear both copies so that checkpoints are deterministic
  if (e == hipSuccess) e = hipMemsetAsync(c.f[0], 0, fbytes, c.stream);
  if (e == hipSuccess) e = hipMemsetAsync(c.f[1], 0, fbytes, c.stream);
  if (e == hipSuccess) {
    lbm::split_table(p->lattice, p->storage).init(c, rho_dev, c.f[0]);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e == hipSuccess && tune && c.path == LB_PATH_SWEEP && p->lattice == LB_D2Q9) {
    // choose the sweep's segment length on this very state, then return to
    // rest equilibrium with both copies cleared as above
    c.cur = 0;
    tune_sweep(c);
    e = hipMemsetAsync(c.f[0], 0, fbytes, c.stream);
    if (e == hipSuccess) e = hipMemsetAsync(c.f[1], 0, fbytes, c.stream);
    if (e == hipSuccess) e = hipMemsetAsync(c.health_flag, 0, sizeof(int), c.stream);
    if (e == hipSuccess) {
      lbm::split_table(p->lattice, p->storage).init(c, rho_dev, c.f[0]);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  }
  if (!staging) (void)hipFree(rho_dev);
  if (e != hipSuccess) {
    lb_free(h);
    return hip_fail(e, "lb_init");
  }
  c.cur = 0;
  c.t = 0;
  *out = h;
  return LB_OK;
}

int fail_with(int code, const char* msg) { return fail(code, msg); }

// Bytes of the lb_moments scratch for a context: rho, mu, h (N*S each), U
// (D*S) and P (D(D+1)/2 * S) doubles.
size_t moments_scratch_bytes(const lb_ctx* h) {
  const Ctx& c = h->c;
  const size_t S = size_t(c.S), N = size_t(c.prm.n_comp), D = size_t(c.D);
  return (3 * N + D + D * (D + 1) / 2) * S * sizeof(double);
}

int moments_impl(lb_ctx* h, void* field_buf, double* rho, double* U, double* mu, double* P, double* mass,
                 double* mom, int64_t* step);

}  // namespace lbm

extern "C" {

int lb_init(const lb_params* p, const double* rho0, void* workspace, size_t workspace_bytes, lb_ctx** out) {
  return lbm::init_impl(p, rho0, workspace, workspace_bytes, nullptr, true, out);
}

int lb_step(lb_ctx* h, int64_t nsteps) {
  if (!h) return fail(LB_EINVAL, "ctx is NULL");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  return advance(h->c, nsteps);
}

int lb_moments(lb_ctx* h, double* rho, double* U, double* mu, double* P, double* mass, double* mom,
               int64_t* step) {
  return lbm::moments_impl(h, nullptr, rho, U, mu, P, mass, mom, step);
}

int lb_moments_noalloc(lb_ctx* h, double* rho, double* U, double* mu, double* P, double* mass, double* mom,
                       int64_t* step) {
  if (!h) return fail(LB_EINVAL, "ctx is NULL");
  const bool fields = rho || U || mu || P;
  void* buf = nullptr;
  if (fields) {
    const size_t need = lbm::moments_scratch_bytes(h);
    if (need > LB_NOALLOC_SCRATCH_BYTES) {
      char msg[200];
      std::snprintf(msg, sizeof msg,
                    "lb_moments_noalloc: the fields need %zu bytes of device scratch, above its static %zu; "
                    "use lb_moments, or ask for mass, mom and step only",
                    need, size_t(LB_NOALLOC_SCRATCH_BYTES));
      return fail(LB_ENOMEM, msg);
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipGetLastError(), "hipGetDevice");
    if (dev != h->c.device) return fail(LB_EINVAL, "lb_moments_noalloc: the context's device is not current");
    hipError_t e = hipSuccess;
    buf = scratch_on(dev, &e);
    if (!buf) return hip_fail(e, "hipGetSymbolAddress of the lb_moments_noalloc scratch");
  }
  return lbm::moments_impl(h, buf, rho, U, mu, P, mass, mom, step);
}

}  // extern "C"

// lb_moments with optional device field buffers of moments_scratch_bytes;
// without them, the field buffers are allocated and freed here.
int lbm::moments_impl(lb_ctx* h, void* field_buf, double* rho, double* U, double* mu, double* P, double* mass,
                      double* mom, int64_t* step) {
  if (!h) return fail(LB_EINVAL, "ctx is NULL");
  Ctx& c = h->c;
  const int N = c.prm.n_comp, D = c.D;
  const size_t S = size_t(c.S);
  const lbm::SplitTable& st = lbm::split_table(c.prm.lattice, c.prm.storage);
  double *d_rho = nullptr, *d_mu = nullptr, *d_h = nullptr, *d_U = nullptr, *d_P = nullptr;
  const bool fields = rho || U || mu || P;
  int rc = LB_OK;
  if (fields) {
    const size_t nP = size_t(D) * (D + 1) / 2;
    hipError_t e = hipSuccess;
    if (field_buf) {
      d_rho = static_cast<double*>(field_buf);
      d_mu = d_rho + N * S;
      d_h = d_mu + N * S;
      d_U = d_h + N * S;
      d_P = d_U + D * S;
    } else {
      e = hipMalloc(&d_rho, N * S * sizeof(double));
      if (e == hipSuccess) e = hipMalloc(&d_mu, N * S * sizeof(double));
      if (e == hipSuccess) e = hipMalloc(&d_h, N * S * sizeof(double));
      if (e == hipSuccess) e = hipMalloc(&d_U, D * S * sizeof(double));
      if (e == hipSuccess) e = hipMalloc(&d_P, nP * S * sizeof(double));
    }
    if (e != hipSuccess) {
      rc = fail(LB_ENOMEM, std::string("lb_moments scratch: ") + hipGetErrorString(e));
    } else {
      st.observe(c, c.f[c.cur], d_rho, d_mu, d_h, d_U, d_P);
      e = hipGetLastError();
      if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d_rho, N * S * 8, hipMemcpyDeviceToHost, c.stream);
      if (e == hipSuccess && mu) e = hipMemcpyAsync(mu, d_mu, N * S * 8, hipMemcpyDeviceToHost, c.stream);
      if (e == hipSuccess && U) e = hipMemcpyAsync(U, d_U, D * S * 8, hipMemcpyDeviceToHost, c.stream);
      if (e == hipSuccess && P) e = hipMemcpyAsync(P, d_P, nP * S * 8, hipMemcpyDeviceToHost, c.stream);
      if (e != hipSuccess) rc = hip_fail(e, "lb_moments");
    }
  }
  double out[lbm::kMaxComp + 3 + 1] = {};  // masses, momentum (D <= 3), flag
  const size_t nout = size_t(lbm::kMaxComp + D + 1);
  int flag = 0;
  if (rc == LB_OK) {
    st.diag(c, c.f[c.cur]);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(out, c.diag_out, nout * sizeof(double), hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, c.health_flag, sizeof(int), hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) rc = hip_fail(e, "lb_moments");
  } else {
    (void)hipStreamSynchronize(c.stream);
  }
  if (fields && !field_buf) {
    (void)hipFree(d_rho);
    (void)hipFree(d_mu);
    (void)hipFree(d_h);
    (void)hipFree(d_U);
    (void)hipFree(d_P);
  }
  if (rc != LB_OK) return rc;
  if (mass)
    for (int k = 0; k < N; ++k) mass[k] = out[k];
  if (mom)
    for (int a = 0; a < D; ++a) mom[a] = out[lbm::kMaxComp + a];
  if (step) *step = c.t;
  if (flag) return fail(LB_ENUMERIC, "a component density became non-finite or <= 0");
  return LB_OK;
}

extern "C" {

int lb_get_f(lb_ctx* h, double* f) {
  if (!h || !f) return fail(LB_EINVAL, "NULL argument");
  Ctx& c = h->c;
  const size_t n = size_t(c.prm.n_comp) * c.Q * size_t(c.S);
  double* d = nullptr;
  HIP_TRY(hipMalloc(&d, n * sizeof(double)));
  lbm::split_table(c.prm.lattice, c.prm.storage).unpull(c, c.f[c.cur], d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "lb_get_f");
  return LB_OK;
}

// State blob: the current population copy, the shift reference (which
// decodes shifted FP16 storage) and the step count.
size_t lb_state_bytes(const lb_ctx* h) {
  if (!h) return 0;
  return h->c.pop_bytes + sizeof(lbm::ShiftRef) + sizeof(int64_t);
}

int lb_get_state(lb_ctx* h, void* host, size_t bytes) {
  if (!h || !host) return fail(LB_EINVAL, "NULL argument");
  Ctx& c = h->c;
  const size_t need = lb_state_bytes(h);
  if (bytes < need) return fail(LB_EINVAL, "buffer too small for the state");
  char* out = static_cast<char*>(host);
  HIP_TRY(hipMemcpyAsync(out, c.f[c.cur], c.pop_bytes, hipMemcpyDeviceToHost, c.stream));
  HIP_TRY(hipStreamSynchronize(c.stream));
  std::memcpy(out + c.pop_bytes, &c.pf.sh, sizeof(lbm::ShiftRef));
  std::memcpy(out + c.pop_bytes + sizeof(lbm::ShiftRef), &c.t, sizeof(int64_t));
  return LB_OK;
}

int lb_set_state(lb_ctx* h, const void* host, size_t bytes) {
  if (!h || !host) return fail(LB_EINVAL, "NULL argument");
  Ctx& c = h->c;
  const size_t need = lb_state_bytes(h);
  if (bytes != need) return fail(LB_EINVAL, "state size does not match this context");
  const char* in = static_cast<const char*>(host);
  HIP_TRY(hipMemcpyAsync(c.f[c.cur], in, c.pop_bytes, hipMemcpyHostToDevice, c.stream));
  HIP_TRY(hipStreamSynchronize(c.stream));
  std::memcpy(&c.pf.sh, in + c.pop_bytes, sizeof(lbm::ShiftRef));
  c.pd.sh = c.pf.sh;
  std::memcpy(&c.t, in + c.pop_bytes + sizeof(lbm::ShiftRef), sizeof(int64_t));
  return LB_OK;
}

int lb_lattice_tables(int32_t lattice, int32_t* Q, int32_t* D, int32_t* v, double* w) {
  int q, d;
  if (lattice_dims(lattice, &q, &d)) return fail(LB_EINVAL, "unknown lattice");
  if (Q) *Q = q;
  if (D) *D = d;
  for (int i = 0; i < q; ++i) {
    int cx, cy, cz;
    double wi;
    switch (lattice) {
      case LB_D1Q3:
        cx = lbm::Lattice<1>::cx(i); cy = lbm::Lattice<1>::cy(i); cz = lbm::Lattice<1>::cz(i);
        wi = lbm::Lattice<1>::w(i);
        break;
      case LB_D2Q9:
        cx = lbm::Lattice<2>::cx(i); cy = lbm::Lattice<2>::cy(i); cz = lbm::Lattice<2>::cz(i);
        wi = lbm::Lattice<2>::w(i);
        break;
      default:
        cx = lbm::Lattice<3>::cx(i); cy = lbm::Lattice<3>::cy(i); cz = lbm::Lattice<3>::cz(i);
        wi = lbm::Lattice<3>::w(i);
        break;
    }
    if (v) {
      v[3 * i] = cx;
      v[3 * i + 1] = cy;
      v[3 * i + 2] = cz;
    }
    if (w) w[i] = wi;
  }
  return LB_OK;
}

int lb_path_in_use(const lb_ctx* h) { return h ? h->c.path : fail(LB_EINVAL, "ctx is NULL"); }

void lb_free(lb_ctx* h) {
  if (!h) return;
  Ctx& c = h->c;
  (void)hipStreamSynchronize(c.stream);
  if (c.owns_ws && c.ws) (void)hipFree(c.ws);
  delete h;
}

const char* lb_strerror(int code) {
  switch (code) {
    case LB_OK: return "success";
    case LB_EINVAL: return "invalid argument";
    case LB_ENOMEM: return "out of memory";
    case LB_ENOTSUP: return "not supported";
    case LB_EDEVICE: return "HIP runtime error";
    case LB_ENUMERIC: return "non-finite or non-positive density";
    default: return "unknown status";
  }
}

const char* lb_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
