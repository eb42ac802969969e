// molt_internal.h -- types shared by the host driver and the HIP kernels of
// libmolt (not part of the public ABI).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "molt.h"

namespace molt {

constexpr int kMaxM = 6;
constexpr int kTuneClasses = 7;  // line length classes n <= 128, 256, ..., 8192 of the shape table

// Coefficients of one line inverse L^{-1} = (I - d^2/alpha^2)^{-1} along one
// axis (Sec. 3.2), built in FP64 on the host.
//  - wl/wr: weights of the centred (M+1)-point stencils of J^L_j and J^R_j,
//    index i <-> node j + i - M/2 (kernel alpha*exp, so the particular
//    solution is (IL + IR)/2).
//  - Non-periodic lines use the same centred stencil with ghost values beyond
//    each end, extrapolated by the degree-M polynomial through the M+1 end
//    nodes; a centred window that leaves the line then interpolates exactly
//    the polynomial of the nearest in-range window, which is the boundary
//    treatment of the oracle.  ghostL[g-1][i]: weight of node i (0..M) for the
//    value at node -g; ghostR[g-1][i]: weight of node n-1-M+i for node n-1+g.
struct LineCoef {
  int32_t n;    // nodes per line
  int32_t N;    // cells per line (n periodic, n-1 otherwise)
  int32_t bc;   // MOLT_BC_*
  int32_t M;    // stencil order
  double nu;    // alpha*h
  double d;     // exp(-nu)
  double mu;    // exp(-nu*N)
  double wl[kMaxM + 1];
  double wr[kMaxM + 1];
  double ghostL[kMaxM / 2][kMaxM + 1];
  double ghostR[kMaxM / 2][kMaxM + 1];
};

// Fixed-point iteration control kept on the device so that queued
// iterations after convergence become no-ops (no host round trip per
// iteration).
struct DevState {
  int open_parts;                 // residual partials of an iteration not yet closed (the block
                                  // count of its P4 x-pass); 0: none pending
  int done;                       // 1: converged or max_iter reached
  int iters;                      // iterations completed in this step
  int max_iter;
  int fixed;                      // >0: never stop early
  double tol;
  double last_resid;
  double mass, energy;
  double mass2;                   // vector model: mass of the second component
};

// thread rows of a y-pass block (a segment is kRG*K rows of 64 columns)
constexpr int kRG = 4;

// Deferred y-pass corrections.  Inside the solver a y-pass scans each
// segment of S rows of a column from zero (its outputs hold the
// segment-local values w_loc) and leaves per (segment, column) seeds: the true
// value is w_loc + 1/2 d^(j - j0s) seedL + 1/2 d^(jls - j) seedR (row j of the
// segment [j0s, jls], d = e^{-nu}).  The next x-pass, which reads those outputs
// anyway, adds the two terms as it loads them, so the y-pass reads its inputs
// once (no totals-then-final double read).
struct YCorr {
  const void* seeds;  // the y-pass's seeds ([comp][field][L,R][segment][column]); nullptr: none
  int nf;             // raw fields of the x-pass that are y-pass outputs (its first nf)
  int nseg, S;        // segments per column, rows per segment
  int ny, nx;         // rows per component, columns
  double nu;          // alpha*h of the y-lines
};

// Arguments of the pass kernels (pointers are device pointers of element type T,
// passed as void* so one struct serves both precisions).
struct PassArgs {
  const void* in[6];
  void* out[3];
  double sigma;    // linear part of f moved to the left-hand side
  double kappa;    // a/s1
  int mode;        // 0: full form (first iteration), 1: increment form
  int bdf2;        // rhs program: 1 -> (4u - u_prev)/3; 2 -> rc0 u + rc1 u_prev (variable steps);
                   // 3 -> (18u - 9u_prev + 2u_prev2)/11 (BDF3)
  double rc0, rc1; // variable-step BDF2 rhs coefficients
  double ushift[2];// u = stored value + ushift, per component: 0 when the fields hold u; the
                   // shifted variable v = u - ushift of Dirichlet steps otherwise
  YCorr corr;      // x-passes: corrections of the preceding deferred y-pass
  // P1 y-pass: residual partials of the previous iteration, closed by the
  // pass's first block before its own work (nullptr: no close here)
  const double* close_part;
  int defer_close; // P4 x-pass: leave its close to the next P1 y-pass or an explicit close
};

// --------------------------------------------------------------------------
// Batched instances: every instance ("slot") advances on its own through the
// phases of its time steps; each tick runs the four line passes once over all
// slots (the rhs/R sweeps for slots in PH_R, one fixed-point iteration for
// slots in PH_IT), then closes iterations and finishes converged steps.
// --------------------------------------------------------------------------
enum SlotPhase { PH_R = 0, PH_IT = 1, PH_IDLE = 2 };

// An FP32 step runs iteration k in FP64 (full form, from the iterate) when
// k % kRestartEvery == 0, in FP32 (increment form) otherwise; the same
// schedule in the single-problem and batched paths.  FP32 rounding of the
// intermediates injects noise relative to the current increments; the part of
// it that lands in nearly neutral modes of the iteration (high in both
// directions, or localized at Neumann ends) is not damped, and after large
// early increments it can stay above the tolerance.  A full-form FP64
// iteration measures the true increment and restarts the recurrence from it.
constexpr int kRestartEvery = 64;

// workspace fields of one problem
// (vector model: every field holds both components; F_E, F_LIN hold the
// reaction and linear parts of the iterate, empty for Cahn-Hilliard; BDF3:
// F_HIST2 the second history, F_STAGE the SDIRK2 stage value, empty otherwise)
enum { F_R = 0, F_DL, F_W, F_A1, F_B1, F_C, F_Q, F_M, F_N, F_HIST, F_E, F_LIN, F_HIST2, F_STAGE, F_COUNT };

struct SlotCtl {  // mutable control of one slot (device)
  int phase;      // SlotPhase
  int step;       // steps completed
  int var;        // coefficient set of the current step: 0 BE, 1 BDF2
  int fp64;       // 1: the slot's next tick runs in the FP64 kernels (always in an FP64
                  // batch; an FP32 slot's R phase, first iteration and restarts)
};

struct SlotDesc {          // constants of one slot, built on the host
  LineCoef cx[2][2];       // [BE, BDF2][alpha1, alpha2] along x
  LineCoef cy[2][2];       // the same along y
  double sigma[2], kappa[2], s1[2], s2[2];
  void* u;                 // the caller's field (u^n in, u^{n+1} out)
  void* fld[F_COUNT];      // workspace fields
  void* tot;               // y-pass segment totals / seeds
  void* jln;               // y-pass periodic closing-cell quadratures
  DevState* st;
  double* rpart;           // residual partials, one per x-pass block
  double* partials;        // mass / energy partials, two per diagnostic block
  molt_step_info* rec;     // nsteps per-step records
  double hx, hy, eps, area;
  double tol;
  int32_t nx, ny, bc, M;
  int32_t stepper, init, nsteps, max_iter;
  int32_t fixed, tlx, vecx, xblocks;  // x-pass: threads per row, 16-byte access, blocks
  int32_t ynth, ynseg, ycols, dblocks;  // y-pass: threads per column, segments, 64-column strips
  int32_t yk;                           // y-pass nodes per thread
  int32_t model, ncomp;                 // MOLT_MODEL_*, field components (1 or 2)
  // FP32 instance with an FP64 shadow: its R phase and the first (full-form)
  // iteration of every step run in the FP64 kernels on these fields, its
  // later iterations in FP32 (the single-problem path does the same)
  int32_t hybrid;
  void* fld64[F_COUNT];
  void* tot64;
  void* jln64;
  void* u64;                            // u^n widened at the start of a step
  void* hist64;                         // u^{n-1} widened (BDF2 steps)
  int32_t tlx64, vecx64, xblocks64;     // FP64 x-pass shape
  int32_t ynth64, ynseg64, yk64;        // FP64 y-pass shape
};

// one block of a batched launch: (slot, block index within the slot)
struct BlkMap {
  int32_t slot, blk;
};

// Optional per-kernel timing with HIP events on the launch stream (off unless
// molt_profile(1) was called).  kind = family * 8 + program.
enum KernelFamily { KF_XPASS = 0, KF_YTOT = 1, KF_YCOMB = 2, KF_YFIN = 3, KF_POINTWISE = 4, KF_OTHER = 5 };
// FP64 launches are counted apart: kind + kProfF64
constexpr int kProfF64 = 48;
constexpr int kProfKinds = 96;
template <typename T>
constexpr int prof_kind(int kind) {
  return kind + (sizeof(T) == 8 ? kProfF64 : 0);
}
void prof_begin(int kind, hipStream_t s);
void prof_end(int kind, hipStream_t s);
// a pair of events for one timed launch of `kind` (both nullptr when that kind
// is not timed); the launch stamps the kernel's own start and end into them
void prof_pair(int kind, hipEvent_t* b, hipEvent_t* e);
extern bool g_prof_on;

// One kernel launch; while kernel timing is on (and `kind` is timed) the
// kernel's start and end are stamped by the dispatch itself
// (hipExtLaunchKernelGGL), so the measured interval is the kernel's alone,
// without the event packets' own processing that an event pair recorded
// around the launch adds.
template <typename... KA, typename... A>
inline void launch_timed(int kind, void (*kern)(KA...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
                         A... args) {
  hipEvent_t b = nullptr, e = nullptr;
  if (g_prof_on) prof_pair(kind, &b, &e);
  hipExtLaunchKernelGGL(kern, grid, block, shmem, s, b, e, 0, args...);
}

}  // namespace molt
