// Internal declarations shared by the library's translation units.
// Not part of the public ABI (that is include/sinkhorn.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/sinkhorn.h"

namespace sk {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;

// One run of Algorithm 1 on K = Prow Pcol^T, as seen by the persistent
// solver.  Device-resident (uploaded into the workspace).
struct SolveDesc {
  const float* Prow;     // n x r, row side (scaling u)
  const float* Pcol;     // m x r, column side (scaling v)
  const float* a;        // n
  const float* b;        // m
  const float* srow;     // n log-scales of Prow or nullptr
  const float* scol;     // m log-scales of Pcol or nullptr
  float* u;              // n: start (warm) / result
  float* v;              // m: result
  float* v2;             // m: second buffer of v (stop test needs v^(k-1))
  float* w;              // r: result Pcol^T v
  float* w2;             // r: second buffer of w
  float* z;              // r: result Prow^T u
  float* slots;          // per-workgroup partial r-vectors, stride slot_stride
  int32_t* members;      // g entries: workgroup index holding each seat
  double* dpart;         // kDpartSlots x g float64 partials (error, flags,
                         // dual sums, weight sums and weight flags)
  unsigned* bar;         // group barrier counter (zeroed before the launch)
  sk_solve_info* info;   // result record
  double tol;
  double eps;
  int64_t n, m;
  int32_t r;
  int32_t g;             // workgroups that run this solve together
  int32_t max_iter;
  int32_t fixed_iter;
  int32_t warm;
  int32_t seat0;         // first seat index of this solve in the launch
  int32_t slot_stride;   // floats between consecutive workgroup slots
  int32_t pad0;
};

// float64 partials per workgroup seat of a solve (SolveDesc::dpart).
constexpr int kDpartSlots = 7;

// Launch-wide control block (zeroed by init_ctl before each launch).
struct LaunchCtl {
  unsigned next_seat;
  unsigned abort_flag;
  unsigned pad[62];
};

// Largest group size (workgroups per solve) the library plans with; it
// bounds workspace sizes independently of the device.
constexpr int kMaxGroup = 2048;

// Largest r of the solver class that handles feature count r (0 if none).
int solver_class_rmax(int r);

// Lanes per feature row of that class (each workgroup's kBlock threads
// cover kBlock / lanes rows at a time; 0 if none).
int solver_class_lanes(int r);

// Maximum number of co-resident workgroups of the solver for feature
// count r (xr != 0: extended-range kernels) on the current device (0 on
// error).
int solver_capacity(int r, int xr);

// Lane layouts of the solver class serving r: writes up to `max` entries
// of (G lanes per row, C float4 per lane, U rows per lane and batch, W
// waves per SIMD) into out (4 ints each) and returns how many the class
// has (variant 0 first: the default).
int solver_layouts(int r, int32_t* out, int max);

// Layout variant in use for the class whose largest r is rmax (the tuning
// table's entry, 0 by default); the solver's class lookups read it.
int solver_layout_variant(int rmax);

// Copy host bytes to device memory with stream-ordered kernel launches
// (the bytes travel as kernel arguments), so the copy can be graph-captured
// and the host buffer may be reused as soon as the call returns.
hipError_t upload_bytes(void* dev, const void* host, size_t nbytes,
                        hipStream_t s);

// Upload `count` solve descriptors (host array) to dev (device array) with
// stream-ordered kernel launches, so the upload can be graph-captured.
hipError_t upload_descs(SolveDesc* dev, const SolveDesc* host, int count,
                        hipStream_t s);

// Run all solves in `dev_descs` (count entries, all with the same r class
// and numeric domain) in one persistent launch.  total_seats = sum of g.
// In the extended range a second launch follows, which resumes only the
// solves the first left for it (see solve.hip); bars (count counters) are
// cleared again for it.
hipError_t launch_solver(const SolveDesc* dev_descs, int count, int r, int xr,
                         int total_seats, int grid, LaunchCtl* ctl, unsigned* bars,
                         hipStream_t s);

// Features (row-scaled Gaussian positive features; log2 values when
// log2_out != 0).
hipError_t launch_features(const float* X, int64_t n, int d, const float* U,
                           int r, double eps, double q, int log2_out,
                           float* Phi, float* logscale, hipStream_t s);

// Batched features over several (X, U) problems.
struct FeatDesc {
  const float* X;
  const float* U;
  float* Phi;
  float* s;
  int64_t n;
  int32_t d, r;
  double eps, q;         // exact parameters: the per-anchor constants are
                         // formed from them in float64 and rounded once
  int32_t log2_out;
  int32_t pad;
  int64_t tile0;         // first row-tile index of this problem
};
// Features of both clouds of a divergence (same anchors): one matrix-core
// launch for d >= 8, else two launches.
hipError_t launch_features_pair(const float* X, int64_t n, const float* Y, int64_t m,
                                int d, const float* U, int r, double eps, double q,
                                int log2_out, float* PhiX, float* sX, float* PhiY,
                                float* sY, hipStream_t s);
hipError_t launch_features_batched(const FeatDesc* host, int count,
                                   FeatDesc* dev_scratch, hipStream_t s);

// Adjoint kernels.  The numeric domain is read on the device from *xr_flag
// (nonzero: extended range) when xr_flag is not null, else from xr.  In the
// extended range a scaling p is [E(n) | M(n)] and an r-vector g is
// [E(r) | M(r)].
hipError_t launch_features_backward(const float* X, int64_t n, int d,
                                    const float* U, int r, const float* Phi,
                                    const float* p1, const float* g1, float c1,
                                    const float* p2, const float* g2, float c2,
                                    const float* p3, const float* g3, float c3,
                                    const float* grad_out, int accumulate,
                                    const int32_t* xr_flag, int xr, float* dX,
                                    hipStream_t s);
hipError_t launch_features_arccos(const float* X, int64_t n, int d, const float* U,
                                  int r, int s_exp, double sigma, double kappa,
                                  float* Phi, float* logscale, hipStream_t s);
size_t anchor_grad_scratch_floats(int r, int d, int64_t n, int64_t m);
hipError_t launch_anchor_grad(const float* X, int64_t n, const float* Y, int64_t m,
                              int d, const float* U, int r, double q,
                              const float* Phix, const float* Phiy,
                              const float* const* u, const float* const* v,
                              const float* const* w, const float* const* z,
                              const float* grad_out, const int32_t* xr_flag,
                              float* scratch, float* dU, hipStream_t s);
hipError_t launch_weight_grad(const float* u1, const float* u2,
                              const float* u3, int64_t n, double eps,
                              const float* grad_out, const int32_t* xr_flag,
                              double* scratch, int scratch_blocks, float* da,
                              hipStream_t s);

// Accelerated Sinkhorn (accel.hip): planned workgroup count, workspace
// bytes for that count, and the persistent launch (linear domain).
int accel_planned_group(int64_t n, int64_t m, int r);
size_t accel_workspace_bytes(int64_t n, int64_t m, int r, int g);
hipError_t launch_accelerated(const float* Prow, const float* Pcol, const float* a,
                              const float* b, const float* srow, const float* scol,
                              float* u, float* v, float* w, float* z, sk_solve_info* info,
                              int32_t* trials, int64_t n, int64_t m, int r, double eps,
                              double tol, int max_iter, int fixed_iter, double L0, void* ws,
                              int g, hipStream_t s);

hipError_t launch_init_ctl(LaunchCtl* ctl, unsigned* bars, int nbars,
                           hipStream_t s);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Launch timing (see profile.hip).  Kinds: 0 solver, 1 features, 2 adjoint.
enum { kProfSolver = 0, kProfFeatures = 1, kProfAdjoint = 2 };
void* prof_begin(int kind, hipStream_t s);
void prof_end(void* token, hipStream_t s);

}  // namespace sk
