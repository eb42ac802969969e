// molt_batch.hip -- batched kernels: the line passes and the step bookkeeping of
// many independent Cahn-Hilliard problems ("slots") in one launch per kernel
// and (stencil order, boundary kind[, x-pass thread granularity]) group.
//
// A tick is: y-pass 1, x-pass 2, y-pass 3, x-pass 4, iteration close, step
// finish, diagnostics, tick end.  A slot in phase PH_R spends its tick on
// R = A1^{-1} A2^{-1} rhs (Sec. 5.1: y(alpha2) of the rhs, x(alpha2), y(alpha1),
// x(alpha1)); a slot in phase PH_IT on one fixed-point iteration (the passes
// P1..P4 of the single-problem path).  When an iteration converges the same
// tick finishes the step (history rotation, u^{n+1}, mass and energy) and the
// tick end moves the slot to the R phase of its next step, or to PH_IDLE.
// Every block finds its (slot, block) in a static map and runs exactly the
// device body of the single-problem kernels with that slot's coefficients,
// so a slot's arithmetic does not depend on the other slots of the batch.
//
// The file is compiled once per precision (MOLT_BATCH_F64 selects double); the
// launchers carry the precision in their names and the host dispatches.
#include "molt_device.h"

#ifdef MOLT_BATCH_F64
#define MOLT_BT double
#define MOLT_BFN(name) name##_f64
#else
#define MOLT_BT float
#define MOLT_BFN(name) name##_f32
#endif

namespace molt {

// A hybrid slot (an FP32 instance with an FP64 shadow) runs its R phase and
// the first (full-form) iteration of each step in the FP64 kernels and the
// later iterations in the FP32 kernels; both are launched every tick and each
// leaves the other's slots alone.
// the precision of a slot's next tick, kept in its control word by whatever
// changes the phase or the iteration count (init, close, tick end), so that a
// kernel of the other precision leaves after reading that one word
__device__ __forceinline__ int slot_fp64_next(const SlotDesc& d, int phase, int iters) {
  if (!d.hybrid) return 1;  // (an unmixed batch is FP64)
  return phase == PH_R || (phase == PH_IT && iters % kRestartEvery == 0) ? 1 : 0;
}
template <typename T>
__device__ __forceinline__ bool slot_mine(const SlotDesc&, const SlotCtl& cc) {
  return cc.fp64 == (sizeof(T) == 8 ? 1 : 0);
}

// 0: full form (the first iteration, and a hybrid slot's FP64 restarts), 1: increment form
template <typename T>
__device__ __forceinline__ int slot_mode(const SlotDesc& d) {
  return (d.hybrid && sizeof(T) == 8) || d.st->iters == 0 ? 0 : 1;
}

// the fields and line-block shapes a slot uses in the kernels of type T
struct SlotView {
  void* const* F;
  void* tot;
  void* jln;
  const void* u;     // u^n as the rhs reads it (a hybrid slot's FP64 rhs: the FP32 field)
  const void* hist;  // u^{n-1} (likewise)
  const void* base;  // the iterate is base + W
  int32_t ynth, ynseg, yk, tlx, vecx, xblocks;
};
template <typename T>
__device__ __forceinline__ SlotView slot_view(const SlotDesc& d) {
  const bool lin = d.init == MOLT_INIT_LINEAR;
  if (sizeof(T) == 8 && d.hybrid)  // first iteration from R or u^n, restarts from the iterate in F_HIST
    return SlotView{d.fld64, d.tot64, d.jln64, d.u, d.fld[F_HIST],
                    d.st->iters == 0 ? (lin ? d.fld64[F_R] : d.u64) : d.fld64[F_HIST],
                    d.ynth64, d.ynseg64, d.yk64, d.tlx64, d.vecx64, d.xblocks64};
  // (a hybrid slot's FP32 iterations run from the re-based first iterate in F_R)
  return SlotView{d.fld, d.tot, d.jln, d.u, d.fld[F_HIST], (lin || d.hybrid) ? d.fld[F_R] : d.u,
                  d.ynth, d.ynseg, d.yk, d.tlx, d.vecx, d.xblocks};
}

// corrections of the deferred y-pass (lines cy, nf swept fields) for the x-pass after it
__device__ __forceinline__ YCorr slot_ycorr(const SlotDesc& d, const SlotView& v, const LineCoef& cy, int nf) {
  YCorr y;
  y.seeds = v.tot;
  y.nf = nf;
  y.nseg = v.ynseg;
  y.S = kRG * v.yk;
  y.ny = d.ny;
  y.nx = d.nx;
  y.nu = cy.nu;
  return y;
}

// arguments of pass `pass` (1..4) of a slot in phase ph (the same fields as
// the single-problem driver uses)
__device__ __forceinline__ PassArgs slot_args(const SlotDesc& d, const SlotView& v, int ph, int pass, int var,
                                              int mode) {
  PassArgs a;
#pragma unroll
  for (int i = 0; i < 6; ++i) a.in[i] = nullptr;
#pragma unroll
  for (int i = 0; i < 3; ++i) a.out[i] = nullptr;
  a.ushift[0] = a.ushift[1] = 0.0;  // batched instances hold u (no Dirichlet walls)
  a.corr.seeds = nullptr;
  a.close_part = nullptr;  // (the batched close is a kernel of its own)
  a.defer_close = 0;
  a.rc0 = a.rc1 = 0.0;
  void* const* F = v.F;
  if (ph == PH_R) {
    a.sigma = 0.0;
    a.kappa = 0.0;
    a.mode = 0;
    a.bdf2 = var;
    if (pass == 1) {
      a.in[0] = v.u;
      a.in[1] = var ? v.hist : v.u;
      a.out[0] = F[F_A1];
    } else if (pass == 2) {
      a.in[0] = F[F_A1];
      a.out[0] = F[F_B1];
    } else if (pass == 3) {
      a.in[0] = F[F_B1];
      a.out[0] = F[F_A1];
    } else {
      a.in[0] = F[F_A1];
      a.out[0] = F[F_R];
    }
  } else {
    a.sigma = d.sigma[var];
    a.kappa = d.kappa[var];
    a.mode = mode;
    a.bdf2 = 0;
    const void* base = v.base;
    const bool vch = d.model == MOLT_MODEL_VCH;
    if (pass == 0) {  // vector model: the pointwise reaction pass
      a.in[0] = base;
      a.in[1] = F[F_W];
      a.in[2] = F[F_DL];
      a.out[0] = F[F_E];
      a.out[1] = F[F_LIN];
    } else if (pass == 1) {
      a.in[0] = vch ? F[F_E] : base;
      a.in[1] = vch ? F[F_LIN] : F[F_W];
      a.in[2] = vch ? nullptr : F[F_DL];
      a.out[0] = F[F_A1];
      a.out[1] = F[F_B1];
    } else if (pass == 2) {
      a.in[0] = F[F_A1];
      a.in[1] = F[F_B1];
      a.in[2] = vch ? F[F_E] : base;
      a.in[3] = vch ? F[F_LIN] : F[F_W];
      a.in[4] = vch ? nullptr : F[F_DL];
      a.out[0] = F[F_C];
      a.out[1] = F[F_Q];
    } else if (pass == 3) {
      a.in[0] = F[F_C];
      a.in[1] = F[F_Q];
      a.out[0] = F[F_M];
      a.out[1] = F[F_N];
    } else {
      a.in[0] = F[F_M];
      a.in[1] = F[F_N];
      a.in[2] = mode ? F[F_DL] : F[F_R];
      a.in[3] = F[F_W];
      a.out[0] = F[F_DL];
      a.out[1] = F[F_W];
    }
  }
  return a;
}

// deferred y-pass `PASS` (1 or 3) with K nodes per thread (segment-local
// scans and segment totals; the combine writes the seeds the x-pass adds)
template <typename T, int K, int M, bool PER, int PASS>
__global__ void MOLT_PASS_ATTR ypass_batch_kernel(const SlotDesc* __restrict__ sd, const SlotCtl* __restrict__ ctl,
                                                  const BlkMap* __restrict__ map) {
  const BlkMap e = map[blockIdx.x];
  const SlotDesc& d = sd[e.slot];
  const SlotCtl cc = ctl[e.slot];
  if (cc.phase == PH_IDLE || !slot_mine<T>(d, cc)) return;
  const SlotView v = slot_view<T>(d);
  // block = (strip bx, segment by, component bz)
  const int bx = e.blk % d.ycols, rest = e.blk / d.ycols;
  const int by = rest % v.ynseg, bz = rest / v.ynseg;
  const size_t fstride = (size_t)d.ny * (size_t)d.nx;
  const int var = cc.var;
  if (cc.phase == PH_R) {
    constexpr int PR = PASS == 1 ? PROG_RHS : PROG_SWEEP;
    const PassArgs a = slot_args(d, v, PH_R, PASS, var, 0);
    const LineCoef& c = d.cy[var][PASS == 1 ? 1 : 0];
    if constexpr (sizeof(T) == 8 && PASS == 1) {
      if (d.hybrid) {  // the FP64 rhs of an FP32 slot reads its FP32 fields
        yloc_body<T, PROG_RHSW, K, M, PER>(c, a, nullptr, d.nx, v.ynth, v.ynseg, fstride, (T*)v.tot, (T*)v.jln, bx,
                                           by, bz);
        return;
      }
    }
    yloc_body<T, PR, K, M, PER>(c, a, nullptr, d.nx, v.ynth, v.ynseg, fstride, (T*)v.tot, (T*)v.jln, bx, by, bz);
  } else {
    DevState* st = d.st;
    if (st->done) return;
    const PassArgs a = slot_args(d, v, PH_IT, PASS, var, slot_mode<T>(d));
    const LineCoef& c = d.cy[var][PASS == 1 ? 0 : 1];
    if constexpr (PASS == 1) {
      if (d.model == MOLT_MODEL_VCH) {
        yloc_body<T, PROG_P1V, K, M, PER>(c, a, st, d.nx, v.ynth, v.ynseg, fstride, (T*)v.tot, (T*)v.jln, bx, by,
                                          bz);
        return;
      }
    }
    constexpr int PI = PASS == 1 ? PROG_P1 : PROG_P3;
    yloc_body<T, PI, K, M, PER>(c, a, st, d.nx, v.ynth, v.ynseg, fstride, (T*)v.tot, (T*)v.jln, bx, by, bz);
  }
}

// y-pass combine of every slot: map block = (slot, strip + ycols * field)
template <typename T>
__global__ void __launch_bounds__(1024) ycomb_batch_kernel(const SlotDesc* __restrict__ sd,
                                                           const SlotCtl* __restrict__ ctl,
                                                           const BlkMap* __restrict__ map, int pass) {
  const BlkMap e = map[blockIdx.x];
  const SlotDesc& d = sd[e.slot];
  const SlotCtl cc = ctl[e.slot];
  if (cc.phase == PH_IDLE || !slot_mine<T>(d, cc)) return;
  const SlotView v = slot_view<T>(d);
  const bool r = cc.phase == PH_R;
  const int F = r ? 1 : 2;
  // block = (strip bx, field f, component b)
  const int bx = e.blk % d.ycols, rest = e.blk / d.ycols;
  const int f = rest % 2, b = rest / 2;
  if (f >= F) return;
  // pass 1: alpha2 in the R phase, alpha1 in an iteration; pass 3 the other way
  const LineCoef& c = d.cy[cc.var][((pass == 1) == r) ? 1 : 0];
  const int ct = (v.ynseg + kCombWaves - 1) / kCombWaves;
  if (ct <= 8)
    ycomb_body<T, 8>(c, r ? nullptr : d.st, d.nx, v.ynseg, kRG * v.yk, F, (T*)v.tot, (const T*)v.jln, bx, f, b);
  else
    ycomb_body<T, 32>(c, r ? nullptr : d.st, d.nx, v.ynseg, kRG * v.yk, F, (T*)v.tot, (const T*)v.jln, bx, f, b);
}

// x-pass `PASS` (2 or 4)
template <typename T, int K, int M, bool PER, int PASS>
__global__ void MOLT_PASS_ATTR xpass_batch_kernel(const SlotDesc* __restrict__ sd, const SlotCtl* __restrict__ ctl,
                                                  const BlkMap* __restrict__ map) {
  __shared__ T smem[XRow<T, K>::ELEMS];  // shared by the pass bodies below
  const BlkMap e = map[blockIdx.x];
  const SlotDesc& d = sd[e.slot];
  const SlotCtl cc = ctl[e.slot];
  if (cc.phase == PH_IDLE || !slot_mine<T>(d, cc)) return;
  const SlotView v = slot_view<T>(d);
  const int var = cc.var;
  const int nlines = d.ny * d.ncomp;  // the components' rows, stacked
  if (cc.phase == PH_R) {
    PassArgs a = slot_args(d, v, PH_R, PASS, var, 0);
    // the y-pass before: the rhs (alpha2) before pass 2, the sweep (alpha1) before pass 4
    a.corr = slot_ycorr(d, v, d.cy[var][PASS == 2 ? 1 : 0], 1);
    xpass_body<T, PROG_SWEEP, K, M, PER>(d.cx[var][PASS == 2 ? 1 : 0], a, nullptr, nlines, v.tlx, nullptr, v.vecx,
                                         e.blk, smem);
  } else {
    DevState* st = d.st;
    if (st->done) return;
    PassArgs a = slot_args(d, v, PH_IT, PASS, var, slot_mode<T>(d));
    // the y-pass before: P1 (alpha1) before pass 2, P3 (alpha2) before pass 4
    a.corr = slot_ycorr(d, v, d.cy[var][PASS == 2 ? 0 : 1], 2);
    if constexpr (PASS == 2) {
      if (d.model == MOLT_MODEL_VCH) {
        xpass_body<T, PROG_P2V, K, M, PER>(d.cx[var][0], a, st, nlines, v.tlx, nullptr, v.vecx, e.blk, smem);
        return;
      }
    }
    constexpr int PI = PASS == 2 ? PROG_P2 : PROG_P4;
    xpass_body<T, PI, K, M, PER>(d.cx[var][PASS == 2 ? 0 : 1], a, st, nlines, v.tlx, PASS == 4 ? d.rpart : nullptr,
                                 v.vecx, e.blk, smem);
  }
}

// iteration close: one block per listed slot
template <typename T>
__global__ void __launch_bounds__(256) close_batch_kernel(const SlotDesc* __restrict__ sd, SlotCtl* ctl,
                                                          const BlkMap* __restrict__ slots) {
  const int slot = slots[blockIdx.x].slot;
  const SlotDesc& d = sd[slot];
  if (ctl[slot].phase != PH_IT) return;
  // (a hybrid slot's FP64 iterations ran the FP64 x-pass and its blocks)
  residual_close_body(d.rpart, (d.hybrid && d.st->iters % kRestartEvery == 0) ? d.xblocks64 : d.xblocks, d.st);
  __syncthreads();  // (thread 0 of the close has counted the iteration)
  if (threadIdx.x == 0) ctl[slot].fp64 = slot_fp64_next(d, PH_IT, d.st->iters);
}

// step finish of converged slots: u^{n-1} <- u^n (the BDF2 history), u^{n+1} = base + W
template <typename T>
__global__ void __launch_bounds__(256) finish_batch_kernel(const SlotDesc* __restrict__ sd,
                                                           const SlotCtl* __restrict__ ctl,
                                                           const BlkMap* __restrict__ map) {
  const BlkMap e = map[blockIdx.x];
  const SlotDesc& d = sd[e.slot];
  if (ctl[e.slot].phase != PH_IT || !d.st->done) return;
  const size_t n = (size_t)d.nx * (size_t)d.ny * (size_t)d.ncomp;
  T* u = (T*)d.u;
  T* h = (T*)d.fld[F_HIST];
  const T* W = (const T*)d.fld[F_W];
  const T* base = (d.init == MOLT_INIT_LINEAR || d.hybrid) ? (const T*)d.fld[F_R] : u;
  for (size_t i = (size_t)e.blk * blockDim.x + threadIdx.x; i < n; i += (size_t)d.dblocks * blockDim.x) {
    const T uo = u[i];
    const T b = base[i];
    h[i] = uo;
    u[i] = b + W[i];
  }
}

#ifndef MOLT_BATCH_F64  // (precision-independent: defined once)
// hybrid slots: u^n (and u^{n-1} for a BDF2 step) widened to FP64 at the
// start of a step, before the FP64 rhs sweeps read them
__global__ void __launch_bounds__(256) widen_batch_kernel(const SlotDesc* __restrict__ sd,
                                                          const SlotCtl* __restrict__ ctl,
                                                          const BlkMap* __restrict__ map) {
  const BlkMap e = map[blockIdx.x];
  const SlotDesc& d = sd[e.slot];
  const SlotCtl cc = ctl[e.slot];
  // (only the first iterate of an init-PREV slot, u^n, is read in FP64 from a
  // copy: the rhs reads the FP32 fields)
  if (!d.hybrid || cc.phase != PH_R || d.init == MOLT_INIT_LINEAR) return;
  const size_t n = (size_t)d.nx * (size_t)d.ny * (size_t)d.ncomp;
  const float* u = (const float*)d.u;
  double* u64 = (double*)d.u64;
  for (size_t i = (size_t)e.blk * blockDim.x + threadIdx.x; i < n; i += (size_t)d.dblocks * blockDim.x)
    u64[i] = (double)u[i];
}

// hybrid slots after an iteration (the tail of a tick, after the close): after
// an FP64 iteration, its iterate re-based into the FP32 base (F_R) and running
// sum and the increment narrowed; before an FP64 restart, the iterate base +
// W in FP64 (F_HIST of the shadow).  The single-problem driver's schedule.
__global__ void __launch_bounds__(256) rebase_batch_kernel(const SlotDesc* __restrict__ sd,
                                                           const SlotCtl* __restrict__ ctl,
                                                           const BlkMap* __restrict__ map) {
  const BlkMap e = map[blockIdx.x];
  const SlotDesc& d = sd[e.slot];
  if (!d.hybrid || ctl[e.slot].phase != PH_IT) return;
  const int it = d.st->iters;
  if (it == 0) return;
  const bool after64 = (it - 1) % kRestartEvery == 0;
  if (!after64 && (it % kRestartEvery != 0 || d.st->done)) return;
  const size_t n = (size_t)d.nx * (size_t)d.ny * (size_t)d.ncomp;
  float* base = (float*)d.fld[F_R];
  float* W = (float*)d.fld[F_W];
  const double* base64 =
      (const double*)(it == 1 ? (d.init == MOLT_INIT_LINEAR ? d.fld64[F_R] : d.u64) : d.fld64[F_HIST]);
  for (size_t i = (size_t)e.blk * blockDim.x + threadIdx.x; i < n; i += (size_t)d.dblocks * blockDim.x) {
    if (after64) {
      const double v = base64[i] + ((const double*)d.fld64[F_W])[i];
      const float b = (float)v;
      base[i] = b;
      W[i] = (float)(v - (double)b);
      ((float*)d.fld[F_DL])[i] = (float)((const double*)d.fld64[F_W])[i];  // full form: DL = W
    } else {
      ((double*)d.fld64[F_HIST])[i] = (double)base[i] + (double)W[i];
    }
  }
}
#endif

template <typename T>
__global__ void __launch_bounds__(256) diag_batch_kernel(const SlotDesc* __restrict__ sd,
                                                         const SlotCtl* __restrict__ ctl,
                                                         const BlkMap* __restrict__ map) {
  const BlkMap e = map[blockIdx.x];
  const SlotDesc& d = sd[e.slot];
  if (ctl[e.slot].phase != PH_IT || !d.st->done) return;
  if (d.model == MOLT_MODEL_VCH)
    diag_vch_body<T>((const T*)d.u, d.nx, d.ny, d.bc, d.hx, d.hy, d.eps, d.partials, e.blk, d.dblocks);
  else
    diag_body<T>((const T*)d.u, d.nx, d.ny, d.bc, d.hx, d.hy, d.eps, d.partials, e.blk, d.dblocks);
}

// vector model: the pointwise reaction pass of slots in an iteration
template <typename T>
__global__ void __launch_bounds__(256) react_batch_kernel(const SlotDesc* __restrict__ sd,
                                                          const SlotCtl* __restrict__ ctl,
                                                          const BlkMap* __restrict__ map) {
  const BlkMap e = map[blockIdx.x];
  const SlotDesc& d = sd[e.slot];
  const SlotCtl cc = ctl[e.slot];
  if (d.model != MOLT_MODEL_VCH || cc.phase != PH_IT || d.st->done || !slot_mine<T>(d, cc)) return;
  const PassArgs a = slot_args(d, slot_view<T>(d), PH_IT, 0, cc.var, slot_mode<T>(d));
  vch_react_body<T>(a, (size_t)d.nx * (size_t)d.ny, (size_t)e.blk * blockDim.x + threadIdx.x,
                    (size_t)d.dblocks * blockDim.x);
}

// tick end, one block per slot: R -> first iteration (state reset); a finished
// step -> mass and energy, the step record, then the next step's R phase or idle
template <typename T>
__global__ void __launch_bounds__(256) tick_end_batch_kernel(const SlotDesc* __restrict__ sd, SlotCtl* ctl,
                                                             const BlkMap* __restrict__ slots) {
  const int slot = slots[blockIdx.x].slot;
  const SlotDesc& d = sd[slot];
  const SlotCtl cc = ctl[slot];
  DevState* st = d.st;
  const int done = cc.phase == PH_IT ? st->done : 0;
  __syncthreads();  // every thread has read the control word before it changes
  if (cc.phase == PH_R) {
    if (threadIdx.x == 0) {
      st->open_parts = 0;
      st->done = 0;
      st->iters = 0;
      st->max_iter = d.max_iter;
      st->fixed = d.fixed;
      st->tol = d.tol;
      st->last_resid = 0.0;
      st->mass = 0.0;
      st->energy = 0.0;
      st->mass2 = 0.0;
      SlotCtl nc = cc;
      nc.phase = PH_IT;
      nc.fp64 = slot_fp64_next(d, PH_IT, 0);
      ctl[slot] = nc;
    }
    return;
  }
  if (cc.phase != PH_IT || !done) return;
  if (d.model == MOLT_MODEL_VCH)
    diag_vch_final_body(d.partials, d.dblocks, d.area, st);
  else
    diag_final_body(d.partials, d.dblocks, d.area, st);
  if (threadIdx.x == 0) {
    const int var = cc.var;
    molt_step_info r;
    r.iters = st->iters;
    r.converged = (d.fixed > 0 || st->last_resid < d.tol) ? 1 : 0;
    r.residual = st->last_resid;
    r.mass = st->mass;
    r.energy = st->energy;
    r.s1 = d.s1[var];
    r.s2 = d.s2[var];
    r.sigma = d.sigma[var];
    r.mass2 = st->mass2;
    d.rec[cc.step] = r;
    SlotCtl nc;
    nc.step = cc.step + 1;
    if (nc.step < d.nsteps) {
      nc.phase = PH_R;
      nc.var = d.stepper == MOLT_BDF2 ? 1 : 0;
    } else {
      nc.phase = PH_IDLE;
      nc.var = var;
    }
    nc.fp64 = slot_fp64_next(d, nc.phase, 0);
    ctl[slot] = nc;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) init_batch_kernel(const SlotDesc* __restrict__ sd, SlotCtl* ctl, int nslots) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += gridDim.x * blockDim.x) {
    SlotCtl c;
    c.phase = sd[i].nsteps > 0 ? PH_R : PH_IDLE;
    c.step = 0;
    c.var = 0;
    c.fp64 = slot_fp64_next(sd[i], c.phase, 0);
    ctl[i] = c;
  }
}

// number of slots not yet idle -> *out
template <typename T>
__global__ void __launch_bounds__(256) count_active_kernel(const SlotCtl* __restrict__ ctl, int nslots, int* out) {
  __shared__ int red[4];
  int c = 0;
  for (int i = threadIdx.x; i < nslots; i += blockDim.x) c += ctl[i].phase != PH_IDLE ? 1 : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
template <typename T, int K, int M, bool PER>
static hipError_t ybatch_m(int pass, const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* map, int nblk,
                           hipStream_t s) {
  const dim3 blk(64, kRG);
  if (pass == 1) hipLaunchKernelGGL((ypass_batch_kernel<T, K, M, PER, 1>), dim3(nblk), blk, 0, s, sd, ctl, map);
  else hipLaunchKernelGGL((ypass_batch_kernel<T, K, M, PER, 3>), dim3(nblk), blk, 0, s, sd, ctl, map);
  return hipGetLastError();
}

template <typename T, int K>
static hipError_t ybatch_k(int M, bool per, int pass, const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* map,
                           int nblk, hipStream_t s) {
  switch (M) {
    case 2: return per ? ybatch_m<T, K, 2, true>(pass, sd, ctl, map, nblk, s)
                       : ybatch_m<T, K, 2, false>(pass, sd, ctl, map, nblk, s);
    case 4: return per ? ybatch_m<T, K, 4, true>(pass, sd, ctl, map, nblk, s)
                       : ybatch_m<T, K, 4, false>(pass, sd, ctl, map, nblk, s);
    case 6: return per ? ybatch_m<T, K, 6, true>(pass, sd, ctl, map, nblk, s)
                       : ybatch_m<T, K, 6, false>(pass, sd, ctl, map, nblk, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t ybatch_t(int K, int M, bool per, int pass, const SlotDesc* sd, const SlotCtl* ctl,
                           const BlkMap* map, int nblk, hipStream_t s) {
  switch (K) {
    case 4: return ybatch_k<T, 4>(M, per, pass, sd, ctl, map, nblk, s);
    case 8: return ybatch_k<T, 8>(M, per, pass, sd, ctl, map, nblk, s);
    case 16:
      if constexpr (sizeof(T) == 4) return ybatch_k<T, 16>(M, per, pass, sd, ctl, map, nblk, s);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

hipError_t MOLT_BFN(launch_batch_y)(int K, int M, bool per, int pass, const SlotDesc* sd, const SlotCtl* ctl,
                                   const BlkMap* map, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  const int kind = prof_kind<MOLT_BT>(KF_YFIN * 8 + (pass == 1 ? PROG_P1 : PROG_P3));
  if (g_prof_on) prof_begin(kind, s);
  const hipError_t e = ybatch_t<MOLT_BT>(K, M, per, pass, sd, ctl, map, nblk, s);
  if (g_prof_on) prof_end(kind, s);
  return e;
}

hipError_t MOLT_BFN(launch_batch_comb)(int pass, const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* map,
                                      int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  const int kind = KF_YCOMB * 8 + (pass == 1 ? PROG_P1 : PROG_P3);
  if (g_prof_on) prof_begin(prof_kind<MOLT_BT>(kind), s);
  hipLaunchKernelGGL((ycomb_batch_kernel<MOLT_BT>), dim3(nblk), dim3(64, kCombWaves), 0, s, sd, ctl, map, pass);
  if (g_prof_on) prof_end(prof_kind<MOLT_BT>(kind), s);
  return hipGetLastError();
}

template <typename T, int K, int M, bool PER>
static hipError_t xbatch_m(int pass, const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* map, int nblk,
                           hipStream_t s) {
  if (pass == 2)
    hipLaunchKernelGGL((xpass_batch_kernel<T, K, M, PER, 2>), dim3(nblk), dim3(256), 0, s, sd, ctl, map);
  else
    hipLaunchKernelGGL((xpass_batch_kernel<T, K, M, PER, 4>), dim3(nblk), dim3(256), 0, s, sd, ctl, map);
  return hipGetLastError();
}

template <typename T, int K>
static hipError_t xbatch_k(int M, bool per, int pass, const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* map,
                           int nblk, hipStream_t s) {
  switch (M) {
    case 2: return per ? xbatch_m<T, K, 2, true>(pass, sd, ctl, map, nblk, s)
                       : xbatch_m<T, K, 2, false>(pass, sd, ctl, map, nblk, s);
    case 4: return per ? xbatch_m<T, K, 4, true>(pass, sd, ctl, map, nblk, s)
                       : xbatch_m<T, K, 4, false>(pass, sd, ctl, map, nblk, s);
    case 6: return per ? xbatch_m<T, K, 6, true>(pass, sd, ctl, map, nblk, s)
                       : xbatch_m<T, K, 6, false>(pass, sd, ctl, map, nblk, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t xbatch_t(int K, int M, bool per, int pass, const SlotDesc* sd, const SlotCtl* ctl,
                           const BlkMap* map, int nblk, hipStream_t s) {
  switch (K) {
    case 4: return xbatch_k<T, 4>(M, per, pass, sd, ctl, map, nblk, s);
    case 8: return xbatch_k<T, 8>(M, per, pass, sd, ctl, map, nblk, s);
    case 16: return xbatch_k<T, 16>(M, per, pass, sd, ctl, map, nblk, s);
    case 32:
      if constexpr (sizeof(T) == 4) return xbatch_k<T, 32>(M, per, pass, sd, ctl, map, nblk, s);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

hipError_t MOLT_BFN(launch_batch_x)(int K, int M, bool per, int pass, const SlotDesc* sd, const SlotCtl* ctl,
                                   const BlkMap* map, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  const int kind = KF_XPASS * 8 + (pass == 2 ? PROG_P2 : PROG_P4);
  if (g_prof_on) prof_begin(prof_kind<MOLT_BT>(kind), s);
  const hipError_t e = xbatch_t<MOLT_BT>(K, M, per, pass, sd, ctl, map, nblk, s);
  if (g_prof_on) prof_end(prof_kind<MOLT_BT>(kind), s);
  return e;
}

// close, step finish, diagnostics and tick end (kind "other_1") of the listed slots
hipError_t MOLT_BFN(launch_batch_tail)(const SlotDesc* sd, SlotCtl* ctl, const BlkMap* slots, int nslots,
                                      const BlkMap* pmap, int npblk, bool close_only, bool hybrid, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  if (g_prof_on) prof_begin(prof_kind<MOLT_BT>(KF_OTHER * 8 + 1), s);
  hipLaunchKernelGGL((close_batch_kernel<MOLT_BT>), dim3(nslots), dim3(256), 0, s, sd, ctl, slots);
#ifndef MOLT_BATCH_F64
  if (hybrid)
    hipLaunchKernelGGL(rebase_batch_kernel, dim3(npblk), dim3(256), 0, s, sd, (const SlotCtl*)ctl, pmap);
#endif
  if (close_only) {
    if (g_prof_on) prof_end(prof_kind<MOLT_BT>(KF_OTHER * 8 + 1), s);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((finish_batch_kernel<MOLT_BT>), dim3(npblk), dim3(256), 0, s, sd, (const SlotCtl*)ctl, pmap);
  hipLaunchKernelGGL((diag_batch_kernel<MOLT_BT>), dim3(npblk), dim3(256), 0, s, sd, (const SlotCtl*)ctl, pmap);
  hipLaunchKernelGGL((tick_end_batch_kernel<MOLT_BT>), dim3(nslots), dim3(256), 0, s, sd, ctl, slots);
  if (g_prof_on) prof_end(prof_kind<MOLT_BT>(KF_OTHER * 8 + 1), s);
  return hipGetLastError();
}

#ifndef MOLT_BATCH_F64
hipError_t launch_batch_widen(const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* pmap, int npblk, hipStream_t s) {
  if (npblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(widen_batch_kernel, dim3(npblk), dim3(256), 0, s, sd, ctl, pmap);
  return hipGetLastError();
}
#endif

hipError_t MOLT_BFN(launch_batch_react)(const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* pmap, int npblk,
                                       hipStream_t s) {
  if (npblk <= 0) return hipSuccess;
  if (g_prof_on) prof_begin(prof_kind<MOLT_BT>(KF_POINTWISE * 8 + PROG_P1V), s);
  hipLaunchKernelGGL((react_batch_kernel<MOLT_BT>), dim3(npblk), dim3(256), 0, s, sd, ctl, pmap);
  if (g_prof_on) prof_end(prof_kind<MOLT_BT>(KF_POINTWISE * 8 + PROG_P1V), s);
  return hipGetLastError();
}

hipError_t MOLT_BFN(launch_batch_init)(const SlotDesc* sd, SlotCtl* ctl, int nslots, hipStream_t s) {
  const int nb = (nslots + 255) / 256;
  hipLaunchKernelGGL((init_batch_kernel<MOLT_BT>), dim3(nb < 1 ? 1 : nb), dim3(256), 0, s, sd, ctl, nslots);
  return hipGetLastError();
}

hipError_t MOLT_BFN(launch_batch_count)(const SlotCtl* ctl, int nslots, int* out, hipStream_t s) {
  hipLaunchKernelGGL((count_active_kernel<MOLT_BT>), dim3(1), dim3(256), 0, s, ctl, nslots, out);
  return hipGetLastError();
}

}  // namespace molt
