// Internal interface between the C ABI (lb_capi.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "lb.h"
#include "physics.hpp"

namespace lbm {

struct Ctx;
// Fused single-kernel steps; nullptr when no such kernel exists for the
// combination.
using FusedStepFn = void (*)(const Ctx&, const void* fin, void* fout);
FusedStepFn fused_step_for(int lattice, int storage, int n_comp);  // tile kernel, D2Q9
FusedStepFn sweep_step_for(int storage, int n_comp);               // strip sweep, D2Q9, nx % 64 == 0
FusedStepFn sweep3d_step_for(int storage, int n_comp);             // plane sweep, D3Q19, nx % 64 == 0, ny % 4 == 0
// Segment lengths of the sweep to time for this context (up to 8, the
// default first) into cand; 0 when the grid is too small to tune.
int sweep_candidates(const Ctx& c, int* cand);

// Choice of the sweep's segment length, made once in lb_init on the freshly
// initialised state (which is restored afterwards): first `warm` steps with
// the default length (the GPU's clocks settle during the first tens of steps
// after a pause, which would otherwise favour whichever candidate runs
// last), then, in each of `passes` passes, for each candidate one step that
// switches to it and steps_per steps between two events on the context's
// stream; then the two candidates with the shortest timings again, in
// rpasses alternating passes of one switching step and rsteps timed steps,
// and the one with the smaller total is kept.
struct SweepTuner {
  static constexpr int kMax = 8;
  static constexpr int warm = 48;
  static constexpr int steps_per = 4;
  static constexpr int passes = 2;
  static constexpr int rsteps = 12;
  static constexpr int rpasses = 2;
};

// Context behind the opaque lb_ctx handle.
struct Ctx {
  lb_params prm;
  int Q = 0, D = 0;
  long long S = 0;
  size_t real_bytes = 0;   // bytes of the working precision
  size_t pop_bytes = 0;    // bytes of one population copy
  hipStream_t stream = nullptr;

  void* ws = nullptr;      // workspace base (device)
  bool owns_ws = false;
  size_t ws_bytes = 0;

  void* f[2] = {nullptr, nullptr};  // population copies, pull storage
  int cur = 0;                      // f[cur] holds the current state
  void* rho_scratch = nullptr;      // [N][S] working precision (split path)
  void* h_scratch = nullptr;        // [N][S] working precision (split path)
  double* diag_partial = nullptr;   // [diag_blocks][K]
  double* diag_out = nullptr;       // [K]: masses (kMaxComp), momentum (D), flag
  int* health_flag = nullptr;       // sticky: 1 once a bad density was seen
  int diag_blocks = 0;

  int device = 0;                   // HIP device current at lb_init
  int64_t t = 0;
  int path = LB_PATH_SPLIT;
  FusedStepFn fused = nullptr;      // kernel of LB_PATH_TILE / LB_PATH_SWEEP
  int sweep_rows = 0;               // segment length of the sweep (0: one-wave default)

  Params<float> pf;
  Params<double> pd;

  template <typename T>
  const Params<T>& params() const;
};

template <>
inline const Params<float>& Ctx::params<float>() const { return pf; }
template <>
inline const Params<double>& Ctx::params<double>() const { return pd; }

struct SplitTable {
  void (*init)(const Ctx&, const double* rho0_dev, void* f);
  void (*step)(const Ctx&, const void* fin, void* fout);
  void (*observe)(const Ctx&, const void* fin, double* rho, double* mu, double* h, double* U, double* P);
  void (*unpull)(const Ctx&, const void* fin, double* out);
  void (*diag)(const Ctx&, const void* fin);
};

const SplitTable& split_table(int lattice, int storage);

// ------------------------------------------------------------ batching ----
// Slot table of the batched kernel (device memory, written by the host).
struct BatchHeader {
  int nslots;  // live slots in the table, in order of first_item
  int items;   // work items (tiles) over all live slots
};

template <typename T>
struct BatchSlot {
  Params<T> p;
  void* f[2];        // population copies; f[t & 1] is current at step t
  long long t_end;   // the slot is stepped while its counter is below this
  int id;            // index of the slot's step counter
  int first_item;    // first work item of the slot
  int tiles_x;       // tiles per row
  int pad;
};

// One configuration of the batched kernel: tile shape, threads per
// workgroup and a launcher for a given grid.
struct BatchKernel {
  int tx, ty, threads;
  // step: one launch advancing every live slot by one step
  void (*step)(const void* slots, const long long* t_now, const BatchHeader* hdr, const int* item_slot, int grid,
               hipStream_t s);
  // advance: counters += 1 for the slots below their target
  void (*advance)(const void* slots, long long* t_now, const BatchHeader* hdr, int max_slots, hipStream_t s);
};

// Candidate configurations for (storage, max components); count in *n.
const BatchKernel* batch_kernels(int storage, int max_comp, int* n);

// Entry points of lb_capi.hip shared with the batch runtime.
int fail_with(int code, const char* msg);  // sets lb_last_error, returns code
int init_impl(const lb_params* p, const double* rho0, void* workspace, size_t workspace_bytes, double* staging,
              bool tune, lb_ctx** out);
size_t moments_scratch_bytes(const lb_ctx* h);
int moments_impl(lb_ctx* h, void* field_buf, double* rho, double* U, double* mu, double* P, double* mass,
                 double* mom, int64_t* step);

}  // namespace lbm

// The opaque handle of the C ABI.
struct lb_ctx {
  lbm::Ctx c;
};
