// Kernel launch interface between the host planner and the HIP kernels.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <string>

#include "aaq_internal.h"
#include "aaqaoa.h"

namespace aaq {

// sets the message aaq_last_error_message returns; returns s
aaq_status set_error(aaq_status s, const std::string& msg);

// host validation of a problem, depth and parameter arrays (no HIP call)
aaq_status validate_call(const aaq_problem* prob, int p, const double* gamma, const double* beta);

// aaq_energy_grad on a given workspace, staging the upload and the results in ordinary
// (pageable) host memory: no device or pinned host allocation
aaq_status energy_grad_pageable(const aaq_problem* prob, int p, const double* gamma, const double* beta,
                                aaq_observable obs, aaq_precision prec, void* d_state, size_t state_bytes,
                                void* d_lambda, size_t lambda_bytes, void* d_ws, size_t ws_bytes, void* stream,
                                double* energy_out, double* dgamma_out, double* dbeta_out, double* norm_out);

// Timing events for the next launches of this host thread (set by the host's per-kernel
// timing, null otherwise).  The first launch takes `start` into its dispatch and every
// launch takes `stop`, so a group of launches is timed from the first kernel's start to
// the last kernel's end by the dispatches themselves, without event packets between them.
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
  bool used = false;
};
LaunchEvents& launch_events();

// every kernel of the library is launched through here
template <class F, class... Args>
inline void launch(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t st, Args... args) {
  LaunchEvents& e = launch_events();
  hipExtLaunchKernelGGL(kernel, grid, block, shm, st, e.start, e.stop, 0u, args...);
  if (e.stop) {
    e.start = nullptr;
    e.used = true;
  }
}

struct LaunchSweep {
  void* psi;
  void* lam;
  const GraphDev* g;
  const int4* terms;
  const void* tab;
  const SwScale* scale;
  double* partial;
  int nslot, T, cmax;
  double amp;
  uint64_t N;  // amplitudes per state (stride between checkpoint buffers)
  SetSpec set;
  SweepProg prog;
  bool two_states;
  bool generic = false;   // take every step from the program at run time
  bool weighted = false;  // integer edge weights (the specialised shapes' weighted copies)
  bool half = false;     // half state: the grid covers the tiles below ntiles / 2
  bool nt = true;        // non-temporal state loads
};

struct LaunchUnits {
  const UnitDesc* units;
  const SweepProg* progs;
  const int32_t* order;
  unsigned char* ws;
  const double* params;
  double* out;
  int32_t* counter;
  int count;
  int out_stride;
  int tabmax;
  void* psi_io;
};

struct LaunchBatch {
  const UnitDesc* units;
  const SweepProg* progs;
  const int32_t* list;  // device list of the group's unit indices
  const int2* wgmap;    // device (unit, tile) of each workgroup of a sweep step
  unsigned char* ws;
  int nlist, max_tiles, wg_count, step, tabmax, route;
  bool two_states, energy;
  uint32_t kind;  // the step's sweep shape (SK_*; SK_GENERIC: the run-time-flag engine)
};

// Tile sizes (log2 amplitudes per workgroup tile) with compiled kernels: sweeps and
// cut dumps for 12 and 13, the persistent unit kernel also for 10.
hipError_t launch_sweep(const LaunchSweep& L, bool dbl, int tile_bits, hipStream_t st);
hipError_t launch_bsweep(const LaunchBatch& L, bool dbl, int tile_bits, hipStream_t st);
hipError_t launch_units(const LaunchUnits& L, bool grad, bool dbl, int tile_bits, int blocks, hipStream_t st);
hipError_t launch_cuts(const GraphDev* g, const int4* terms, int T, int use_terms, const SetSpec& S, int arr,
                       int32_t* out, bool dbl, int tile_bits, hipStream_t st);
hipError_t launch_bsweep_out(const LaunchBatch& L, double* out, int out_stride, bool grad, bool dbl, hipStream_t st);
hipError_t launch_tables(const double* gamma, const double* beta, int p, int cmax, void* tab, const SweepProg* progs,
                         int nsweep, const SetSpec* sets, int nsets, SwScale* scales, bool dbl, hipStream_t st);
hipError_t launch_plan_tables(const LaunchUnits& L, int p, bool dbl, hipStream_t st);
// light-cone units: copy the shared parameters [np] into every unit row; sum the unit
// output rows [count][stride] in unit order (column 1, the norm, is averaged)
// final-state sampling: block sums of |psi|^2, their prefix in bitstring order, one
// inverse-CDF draw per uniform number (one wave per shot), cut values, best / mean cut
hipError_t launch_sample(const void* psi, int n, int lb, double* bsum, double* cum, double* ssum, const uint64_t* flips,
                         const double* uniform, int shots, const GraphDev* g, const int4* cost_terms, uint64_t* samples,
                         int32_t* cuts, double* stats, bool dbl, hipStream_t st);
hipError_t launch_lc_bcast(const double* params, int np, double* rows, int count, hipStream_t st);
hipError_t launch_lc_sum(const double* rows, int count, int stride, double* out, hipStream_t st);
// fixed-order sums of per-tile partials; stage holds nout * kReduceChunks doubles
constexpr int kReduceChunks = 32;
hipError_t launch_reduce(const double* partial, const void* src, const int32_t* src_begin, double* stage, double* out,
                         int nout, hipStream_t st);
hipError_t launch_zz_pass(const void* psi, uint64_t N, int i, int j, const double* scale, const uint64_t* flips,
                          double* partial, int blocks, bool dbl, hipStream_t st);

// per-instantiation entry points (defined by AAQ_INSTANTIATE_* in aaq_inst_*.hip)
#define AAQ_DECLARE_UNITS(SUF) hipError_t launch_units_##SUF(const LaunchUnits& L, bool grad, int blocks, hipStream_t st);
#define AAQ_DECLARE_SWEEPS(SUF)                                                                            \
  hipError_t launch_sweep_##SUF(const LaunchSweep& L, hipStream_t st);                                     \
  hipError_t launch_bsweep_##SUF(const LaunchBatch& L, hipStream_t st);                                    \
  hipError_t launch_cuts_##SUF(const GraphDev* g, const int4* terms, int T, int use_terms, const SetSpec& S, int arr, \
                               int32_t* out, hipStream_t st);
AAQ_DECLARE_UNITS(f10)
AAQ_DECLARE_UNITS(f12)
AAQ_DECLARE_UNITS(f13)
AAQ_DECLARE_UNITS(d10)
AAQ_DECLARE_UNITS(d12)
AAQ_DECLARE_UNITS(d13)
AAQ_DECLARE_SWEEPS(f12)
AAQ_DECLARE_SWEEPS(f13)
AAQ_DECLARE_SWEEPS(d12)
AAQ_DECLARE_SWEEPS(d13)

// RedSrc layout mirrored on the host
struct RedSrcHost {
  int64_t off;
  int32_t count;
  int32_t out;
  double scale;
};

}  // namespace aaq
