// molt_kernels.hip -- HIP kernels (gfx950 / CDNA4) of one problem: the line
// pass kernels, the fused y-pass, pointwise and bookkeeping kernels, and
// their launchers.  The device bodies live in molt_device.h.
//
// The file is compiled four times, once per precision (MOLT_PREC_F64 selects
// double) and pass direction (MOLT_PART_X: x-passes and the shape table;
// MOLT_PART_Y: y-passes and the pointwise kernels), so the template-heavy
// parts build in parallel; the launchers carry the precision in their names
// and the host dispatches.
#include "molt_device.h"

#ifdef MOLT_PREC_F64
#define MOLT_KT double
#define MOLT_KFN(name) name##_f64
#else
#define MOLT_KT float
#define MOLT_KFN(name) name##_f32
#endif
#if !defined(MOLT_PART_X) && !defined(MOLT_PART_Y)
#error "define MOLT_PART_X or MOLT_PART_Y"
#endif
#if defined(MOLT_PART_X) && !defined(MOLT_PREC_F64)
#define MOLT_PART_COMMON 1  // precision-independent helpers: one translation unit only
#endif

namespace molt {

// helpers defined once (MOLT_PART_COMMON) and used by every part
int xpass_max_n(int prec);
int xpass_pick_k(int n, int prec);
int ypass_pick_k(int n, int prec);
int xpass_tl(int n, int K);
int diag_blocks(size_t n);

template <typename T>
__global__ void __launch_bounds__(1024) residual_close_kernel(const double* partials, DevState* st) {
  (void)residual_close_pending(partials, st);
}

template <typename T, int PI, int K, int M, bool PER, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(MOLT_OCC)))
xpass_kernel(const LineCoef c, const PassArgs a, DevState* st, int nlines, int TL, double* rpart, int vec) {
  __shared__ T smem[ProgOf<PI, T>::type::F * XRow<T, K, BS>::PADDED];
  // consecutive blocks are dispatched round-robin over the 8 XCDs: give each
  // XCD a contiguous range of rows, so that the rows of one y-pass segment
  // (which share its seed rows) read them through one XCD's L2
  const int g = gridDim.x, b = blockIdx.x;
  // (P2 and P4 at 4096^2: 100 -> 92 us and 98 -> 87 us)
  const int bx = (g % 8 == 0) ? (b % 8) * (g / 8) + b / 8 : b;
  // (before the body: a block that returns early must not skip it; done
  // does not change during the pass)
  if (rpart != nullptr && b == 0 && threadIdx.x == 0 && !st->done) st->open_parts = g;
  xpass_body<T, PI, K, M, PER, BS>(c, a, st, nlines, TL, rpart, vec, bx, smem);
}

template <typename T, int PI, int K, int M, bool PER>
__global__ void MOLT_PASS_ATTR ytot_kernel(const LineCoef c, const PassArgs a, DevState* st, int nx, int nth,
                                           int nseg, size_t fstride, T* agg, T* jlnb) {
  ytot_body<T, PI, K, M, PER>(c, a, st, nx, nth, nseg, fstride, agg, jlnb, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T, int CTMAX>
__global__ void __launch_bounds__(1024) ycomb_kernel(const LineCoef c, DevState* st, int nx, int nth, int K, int F,
                                                     T* tot, const T* jlnb) {
  ycomb_body<T, CTMAX>(c, st, nx, nth, K, F, tot, jlnb, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T, int PI, int K, int M, bool PER>
__global__ void MOLT_PASS_ATTR yfin_kernel(const LineCoef c, const PassArgs a, DevState* st, int nx, int nth,
                                           int nseg, size_t fstride, const T* seeds) {
  yfin_body<T, PI, K, M, PER>(c, a, st, nx, nth, nseg, fstride, seeds, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T, int PI, int K, int M, bool PER>
__global__ void MOLT_PASS_ATTR yloc_kernel(const LineCoef c, const PassArgs a, DevState* st, int nx, int nth,
                                           int nseg, size_t fstride, T* agg, T* jlnb) {
  yloc_body<T, PI, K, M, PER>(c, a, st, nx, nth, nseg, fstride, agg, jlnb, blockIdx.x, blockIdx.y, blockIdx.z);
}

#ifdef MOLT_PART_COMMON
__global__ void __launch_bounds__(256) zero_ints_kernel(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}
#endif

// pointwise program with the identity in place of the sweep (the y-direction
// of a one-dimensional problem)
template <typename T, int PI>
__global__ void __launch_bounds__(256) pointwise_kernel(const PassArgs a, DevState* st, size_t nelem) {
  using P = typename ProgOf<PI, T>::type;
  constexpr int F = P::F, E = P::E, NR = P::NR, NO = P::NO;
  if (st != nullptr && st->done) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nelem; i += (size_t)gridDim.x * blockDim.x) {
    T r[NR], s[F], x[E > 0 ? E : 1], o[NO];
    load_raw<T, P>(a, i, r);
    P::sin(a, r, s);
    if constexpr (E > 0) P::ext(a, r, x);
    P::fin(a, s, x, o);
#pragma unroll
    for (int f = 0; f < NO; ++f) ((T*)a.out[f])[i] = o[f];
  }
}

// --------------------------------------------------------------------------
// step bookkeeping
// --------------------------------------------------------------------------
#ifdef MOLT_PART_COMMON
__global__ void state_init_kernel(DevState* st, double tol, int max_iter, int fixed) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->open_parts = 0;
    st->done = 0;
    st->iters = 0;
    st->max_iter = max_iter;
    st->fixed = fixed;
    st->tol = tol;
    st->last_resid = 0.0;
    st->mass = 0.0;
    st->energy = 0.0;
    st->mass2 = 0.0;
  }
}
#endif

template <typename T>
__global__ void __launch_bounds__(256) copy_kernel(T* dst, const T* src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// u^{n+1} = base + W
template <typename T>
__global__ void __launch_bounds__(256) finalize_kernel(T* u, const T* base, const T* W, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    u[i] = base[i] + W[i];
}

template <typename T>
__global__ void __launch_bounds__(256) diag_kernel(const T* u, int nx, int ny, int bc, double hx, double hy,
                                                   double eps, double* partials) {
  diag_body<T>(u, nx, ny, bc, hx, hy, eps, partials, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) diag_vch_kernel(const T* u, int nx, int ny, int bc, double hx, double hy,
                                                       double eps, double* partials) {
  diag_vch_body<T>(u, nx, ny, bc, hx, hy, eps, partials, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) diag_vch_final_kernel(const double* partials, int nblocks, double area,
                                                             DevState* st) {
  diag_vch_final_body(partials, nblocks, area, st);
}

// vector model: (e, lin) of both components (n nodes per component)
template <typename T>
__global__ void __launch_bounds__(256) vch_react_kernel(const PassArgs a, DevState* st, size_t n) {
  if (st != nullptr && st->done) return;
  vch_react_body<T>(a, n, (size_t)blockIdx.x * blockDim.x + threadIdx.x, (size_t)gridDim.x * blockDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) maxdiff_kernel(const T* a, const T* b, size_t n, double* partials) {
  maxdiff_body<T>(a, b, n, partials, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(64) maxdiff_final_kernel(const double* partials, int nb, double* out) {
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += 64) m = fmax(m, partials[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off));
  if (threadIdx.x == 0) out[0] = m;
}

template <typename T>
__global__ void __launch_bounds__(256) diag_final_kernel(const double* partials, int nblocks, double area,
                                                         DevState* st) {
  diag_final_body(partials, nblocks, area, st);
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
#ifdef MOLT_PART_COMMON
static int pick_kx(int n, int prec) {
  const int ks[4] = {4, 8, 16, 32};
  const int kmax = prec == MOLT_F64 ? 16 : 32;
  for (int i = 0; i < 4; ++i)
    if (ks[i] <= kmax && n <= 256 * ks[i]) return ks[i];
  return 0;
}

int xpass_max_n(int prec) { return prec == MOLT_F64 ? 4096 : 8192; }

// --------------------------------------------------------------------------
// Line-block shapes: nodes per thread along x (kx) and along y (ky) per line
// length class (n <= 128, 256, ..., 8192) and precision; process-wide, set by
// molt_tune_set or measured by molt_autotune.  Defaults: the smallest kx that
// fits a line in one 256-thread block, except FP32 lines of 8192 nodes, whose
// iteration passes spill registers at 32 nodes per thread (they take 16 in
// 512-thread rows); ky = 16 (FP32) / 8 (FP64).
// --------------------------------------------------------------------------
static int g_kx[2][kTuneClasses] = {{4, 4, 4, 4, 8, 16, 16}, {4, 4, 4, 4, 8, 16, 16}};
static int g_ky[2][kTuneClasses] = {{8, 8, 8, 8, 8, 8, 8}, {16, 16, 16, 16, 16, 16, 16}};

int tune_class(int n) {
  int c = 0;
  while (c < kTuneClasses - 1 && n > (128 << c)) ++c;
  return c;
}

bool tune_valid(int prec, int cls, int kx, int ky) {
  if (cls < 0 || cls >= kTuneClasses || (prec != MOLT_F64 && prec != MOLT_F32)) return false;
  const bool kx_ok = kx == 4 || kx == 8 || kx == 16 || (kx == 32 && prec == MOLT_F32);
  const bool ky_ok = ky == 4 || ky == 8 || (ky == 16 && prec == MOLT_F32);
  const int nmax = cls == kTuneClasses - 1 ? xpass_max_n(prec) : (128 << cls);
  // rows of 512 threads only for lines longer than 2048 nodes (the batched
  // kernels, which run 256-thread blocks, then take the smallest 256-thread kx)
  const int row_threads = cls >= 5 ? 512 : 256;
  return kx_ok && ky_ok && nmax <= row_threads * kx;
}

void tune_get(int prec, int cls, int* kx, int* ky) {
  *kx = g_kx[prec == MOLT_F32][cls];
  *ky = g_ky[prec == MOLT_F32][cls];
}

void tune_set(int prec, int cls, int kx, int ky) {
  g_kx[prec == MOLT_F32][cls] = kx;
  g_ky[prec == MOLT_F32][cls] = ky;
}

// launch shapes shared with the batched driver
int xpass_pick_k(int n, int prec) {
  const int k = g_kx[prec == MOLT_F32][tune_class(n)];
  return n <= 512 * k ? k : pick_kx(n, prec);
}
// the batched kernels run 256-thread blocks: a row gets at most 256 threads
int xpass_pick_k256(int n, int prec) {
  const int k = g_kx[prec == MOLT_F32][tune_class(n)];
  return n <= 256 * k ? k : pick_kx(n, prec);
}
int ypass_pick_k(int n, int prec) { return g_ky[prec == MOLT_F32][tune_class(n)]; }
// the largest block counts any shape of the table can give (workspace sizing)
int ypass_max_segments(int n) {
  const int nth = (n + 3) / 4;
  return (nth + kRG - 1) / kRG;
}
int xpass_min_k(int n, int prec) { return pick_kx(n, prec); }
int xpass_tl(int n, int K) {
  const int need = (n + K - 1) / K;
  return need <= 64 ? 64 : (need <= 128 ? 128 : (need <= 256 ? 256 : 512));
}
void ypass_shape(int prec, int n, int* nth, int* nseg) {
  const int K = ypass_pick_k(n, prec);
  *nth = (n + K - 1) / K;
  *nseg = (*nth + kRG - 1) / kRG;
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_ints_kernel, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// The FP64 shadow of an FP32 step: its inputs widened, and the iterate after
// the FP64 first iteration re-based for the FP32 increment iterations.
__global__ void __launch_bounds__(256) widen_kernel(double* dst, const float* src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

// Before an FP64 restart iteration: the iterate base32 + W32 in FP64 (unless
// the step has converged)
__global__ void __launch_bounds__(256) iterate64_kernel(double* v64, const float* base32, const float* W32,
                                                        const DevState* st, size_t n) {
  if (st->done) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v64[i] = (double)base32[i] + (double)W32[i];
}

static dim3 grid_elems(size_t n) {
  size_t b = (n + 255) / 256;
  return dim3((unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b)));
}
hipError_t launch_widen(void* dst64, const void* src32, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(widen_kernel, grid_elems(n), dim3(256), 0, s, (double*)dst64, (const float*)src32, n);
  return hipGetLastError();
}
hipError_t launch_iterate64(void* v64, const void* base32, const void* W32, const DevState* st, size_t n,
                            hipStream_t s) {
  hipLaunchKernelGGL(iterate64_kernel, grid_elems(n), dim3(256), 0, s, (double*)v64, (const float*)base32,
                     (const float*)W32, st, n);
  return hipGetLastError();
}

size_t ypass_tot_elems(int prec, int n, int nx, int batch) {
  (void)prec;
  const int K = 4;  // the smallest ky: room for every shape
  const int nth = (n + K - 1) / K;
  const int nseg = (nth + kRG - 1) / kRG;
  return (size_t)2 * 2 * nseg * nx * batch;  // F <= 2 fields, 2 directions, one entry per segment
}

// the close of an iteration still pending (no-op when none is)
__global__ void __launch_bounds__(1024) close_pending_kernel(const double* partials, DevState* st) {
  (void)residual_close_pending(partials, st);
}
hipError_t launch_close_pending(const double* rpart, DevState* st, hipStream_t s) {
  launch_timed(KF_OTHER * 8, close_pending_kernel, dim3(1), dim3(1024), 0, s, rpart, st);
  return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, double tol, int max_iter, int fixed, hipStream_t s) {
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, st, tol, max_iter, fixed);
  return hipGetLastError();
}

int diag_blocks(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  return (int)(b < 1 ? 1 : b);
}
#endif  // MOLT_PART_COMMON

#ifdef MOLT_PART_X
// 16-byte vector access is used when every field pointer is 16-byte aligned and
// rows are a whole number of 16-byte words
template <typename T, int PI>
static int can_vec(const PassArgs& a, int n) {
  using P = typename ProgOf<PI, T>::type;
  if ((n * (int)sizeof(T)) % 16 != 0) return 0;
  for (int f = 0; f < P::NR + Late<P>::n; ++f)
    if (((uintptr_t)a.in[f]) % 16 != 0) return 0;
  for (int f = 0; f < P::NO; ++f)
    if (((uintptr_t)a.out[f]) % 16 != 0) return 0;
  return 1;
}

template <typename T, int PI, int K>
static hipError_t xpass_k(const LineCoef& c, const PassArgs& a, DevState* st, int nlines, double* rpart, hipStream_t s) {
  const int vec = can_vec<T, PI>(a, c.n);
  // threads per line: 64, 128 or 256, so that 256/TL rows tile the block exactly
  const int TL = xpass_tl(c.n, K);
  const int BS = TL > 256 ? 512 : 256;  // rows of 512 threads get a block of their own
  const int lpb = BS / TL;
  dim3 grid((nlines + lpb - 1) / lpb);
  const int kind = prof_kind<MOLT_KT>(KF_XPASS * 8 + prog_slot(PI));
  const bool per = c.bc == MOLT_BC_PERIODIC;
#define MOLT_XL(MM, PP)                                                                                          \
  do {                                                                                                          \
    if (BS == 512)                                                                                              \
      launch_timed(kind, xpass_kernel<T, PI, K, MM, PP, 512>, grid, dim3(512), 0, s, c, a, st, nlines, TL, rpart, \
                   vec);                                                                                        \
    else                                                                                                        \
      launch_timed(kind, xpass_kernel<T, PI, K, MM, PP, 256>, grid, dim3(256), 0, s, c, a, st, nlines, TL, rpart, \
                   vec);                                                                                        \
  } while (0)
  switch (c.M) {
    case 2: if (per) MOLT_XL(2, true); else MOLT_XL(2, false); break;
    case 4: if (per) MOLT_XL(4, true); else MOLT_XL(4, false); break;
    case 6: if (per) MOLT_XL(6, true); else MOLT_XL(6, false); break;
    default: return hipErrorInvalidValue;
  }
#undef MOLT_XL
  if (rpart != nullptr && !a.defer_close) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_timed(prof_kind<MOLT_KT>(KF_OTHER * 8), residual_close_kernel<T>, dim3(1), dim3(1024), 0, s,
                 (const double*)rpart, st);
  }
  return hipGetLastError();
}

template <typename T, int PI>
static hipError_t xpass_t(const LineCoef& c, const PassArgs& a, DevState* st, int nlines, double* rpart, hipStream_t s,
                          int prec) {
  int k = xpass_pick_k(c.n, prec);
  // the FP64 iteration passes (several fields per node) spill registers at 16
  // nodes per thread; they take 8 in rows of up to 512 threads
  if (sizeof(T) == 8 && k == 16 && prog_slot(PI) != PROG_SWEEP && prog_slot(PI) != PROG_RHS && c.n <= 512 * 8) k = 8;
  switch (k) {
    case 4: return xpass_k<T, PI, 4>(c, a, st, nlines, rpart, s);
    case 8: return xpass_k<T, PI, 8>(c, a, st, nlines, rpart, s);
    case 16: return xpass_k<T, PI, 16>(c, a, st, nlines, rpart, s);
    case 32:
      if constexpr (sizeof(T) == 4) return xpass_k<T, PI, 32>(c, a, st, nlines, rpart, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t MOLT_KFN(launch_xpass)(int prog, const LineCoef& c, const PassArgs& a, DevState* st, int nlines,
                                  double* rpart, hipStream_t s) {
  constexpr int prec = sizeof(MOLT_KT) == 8 ? MOLT_F64 : MOLT_F32;
  switch (prog) {
    case PROG_SWEEP: return xpass_t<MOLT_KT, PROG_SWEEP>(c, a, st, nlines, rpart, s, prec);
    case PROG_RHS: return xpass_t<MOLT_KT, PROG_RHS>(c, a, st, nlines, rpart, s, prec);
    case PROG_P2: return xpass_t<MOLT_KT, PROG_P2>(c, a, st, nlines, rpart, s, prec);
    case PROG_P4: return xpass_t<MOLT_KT, PROG_P4>(c, a, st, nlines, rpart, s, prec);
    case PROG_P2V: return xpass_t<MOLT_KT, PROG_P2V>(c, a, st, nlines, rpart, s, prec);
#ifdef MOLT_PREC_F64
    case PROG_P2F: return xpass_t<MOLT_KT, PROG_P2F>(c, a, st, nlines, rpart, s, prec);
    case PROG_P4F: return xpass_t<MOLT_KT, PROG_P4F>(c, a, st, nlines, rpart, s, prec);
    case PROG_RHSW: return xpass_t<MOLT_KT, PROG_RHSW>(c, a, st, nlines, rpart, s, prec);
    case PROG_P4R: return xpass_t<MOLT_KT, PROG_P4R>(c, a, st, nlines, rpart, s, prec);
#endif
  }
  return hipErrorInvalidValue;
}
#endif  // MOLT_PART_X

#ifdef MOLT_PART_Y

// deferred: the single-read y-pass (yloc, then the combine's seeds for the
// next x-pass); otherwise totals, combine and final scans (final outputs)
template <typename T, int PI, int K, int M, bool PER>
static hipError_t ypass_km(const LineCoef& c, const PassArgs& a, DevState* st, int nx, int batch, T* tot, T* jln,
                           bool deferred, hipStream_t s) {
  using P = typename ProgOf<PI, T>::type;
  const int nth = (c.n + K - 1) / K;
  const int nseg = (nth + kRG - 1) / kRG;
  const size_t fstride = (size_t)c.n * nx;
  dim3 blk(64, kRG);
  dim3 grid((nx + 63) / 64, nseg, batch);
  hipError_t e;
  if (deferred) {
    launch_timed(prof_kind<MOLT_KT>(KF_YFIN * 8 + prog_slot(PI)), yloc_kernel<T, PI, K, M, PER>, grid, blk, 0, s, c, a, st, nx,
                 nth, nseg, fstride, tot, jln);
  } else {
    launch_timed(prof_kind<MOLT_KT>(KF_YTOT * 8 + prog_slot(PI)), ytot_kernel<T, PI, K, M, PER>, grid, blk, 0, s, c, a, st, nx,
                 nth, nseg, fstride, tot, jln);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the combine runs over segments of kRG*K rows
  const int ct = (nseg + kCombWaves - 1) / kCombWaves;
  const dim3 cgrid((nx + 63) / 64, P::F, batch), cblk(64, kCombWaves);
  const int S = kRG * K;
  const int ckind = prof_kind<MOLT_KT>(KF_YCOMB * 8 + prog_slot(PI));
  if (ct <= 8)
    launch_timed(ckind, ycomb_kernel<T, 8>, cgrid, cblk, 0, s, c, st, nx, nseg, S, (int)P::F, tot, (const T*)jln);
  else if (ct <= 16)
    launch_timed(ckind, ycomb_kernel<T, 16>, cgrid, cblk, 0, s, c, st, nx, nseg, S, (int)P::F, tot, (const T*)jln);
  else if (ct <= 32)
    launch_timed(ckind, ycomb_kernel<T, 32>, cgrid, cblk, 0, s, c, st, nx, nseg, S, (int)P::F, tot, (const T*)jln);
  else
    return hipErrorInvalidValue;
  e = hipGetLastError();
  if (e != hipSuccess || deferred) return e;
  launch_timed(prof_kind<MOLT_KT>(KF_YFIN * 8 + prog_slot(PI)), yfin_kernel<T, PI, K, M, PER>, grid, blk, 0, s, c, a, st, nx,
               nth, nseg, fstride, (const T*)tot);
  return hipGetLastError();
}

template <typename T, int PI, int K>
static hipError_t ypass_k(const LineCoef& c, const PassArgs& a, DevState* st, int nx, int batch, void* tot, void* jln,
                          bool deferred, hipStream_t s) {
  const bool per = c.bc == MOLT_BC_PERIODIC;
  switch (c.M) {
    case 2: return per ? ypass_km<T, PI, K, 2, true>(c, a, st, nx, batch, (T*)tot, (T*)jln, deferred, s)
                       : ypass_km<T, PI, K, 2, false>(c, a, st, nx, batch, (T*)tot, (T*)jln, deferred, s);
    case 4: return per ? ypass_km<T, PI, K, 4, true>(c, a, st, nx, batch, (T*)tot, (T*)jln, deferred, s)
                       : ypass_km<T, PI, K, 4, false>(c, a, st, nx, batch, (T*)tot, (T*)jln, deferred, s);
    case 6: return per ? ypass_km<T, PI, K, 6, true>(c, a, st, nx, batch, (T*)tot, (T*)jln, deferred, s)
                       : ypass_km<T, PI, K, 6, false>(c, a, st, nx, batch, (T*)tot, (T*)jln, deferred, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int PI>
static hipError_t ypass_t(const LineCoef& c, const PassArgs& a, DevState* st, int nx, int batch, void* tot, void* jln,
                          bool deferred, hipStream_t s) {
  switch (ypass_pick_k(c.n, sizeof(T) == 8 ? MOLT_F64 : MOLT_F32)) {
    case 4: return ypass_k<T, PI, 4>(c, a, st, nx, batch, tot, jln, deferred, s);
    case 8: return ypass_k<T, PI, 8>(c, a, st, nx, batch, tot, jln, deferred, s);
    case 16:
      if constexpr (sizeof(T) == 4) return ypass_k<T, PI, 16>(c, a, st, nx, batch, tot, jln, deferred, s);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

hipError_t MOLT_KFN(launch_ypass)(int prog, const LineCoef& c, const PassArgs& a, DevState* st, int nx, int batch,
                                  void* tot, void* jln, bool deferred, hipStream_t s) {
  switch (prog) {
    case PROG_SWEEP: return ypass_t<MOLT_KT, PROG_SWEEP>(c, a, st, nx, batch, tot, jln, deferred, s);
    case PROG_RHS: return ypass_t<MOLT_KT, PROG_RHS>(c, a, st, nx, batch, tot, jln, deferred, s);
#ifdef MOLT_PREC_F64
    case PROG_RHSW: return ypass_t<MOLT_KT, PROG_RHSW>(c, a, st, nx, batch, tot, jln, deferred, s);
#endif
    case PROG_P1: return ypass_t<MOLT_KT, PROG_P1>(c, a, st, nx, batch, tot, jln, deferred, s);
    case PROG_P3: return ypass_t<MOLT_KT, PROG_P3>(c, a, st, nx, batch, tot, jln, deferred, s);
    case PROG_P1V: return ypass_t<MOLT_KT, PROG_P1V>(c, a, st, nx, batch, tot, jln, deferred, s);
  }
  return hipErrorInvalidValue;
}

static dim3 grid_1d(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t MOLT_KFN(launch_pointwise)(int prog, const PassArgs& a, DevState* st, size_t nelem, hipStream_t s) {
  dim3 g = grid_1d(nelem);
  const int kind = prof_kind<MOLT_KT>(KF_POINTWISE * 8 + prog);
  if (prog == PROG_P1) launch_timed(kind, pointwise_kernel<MOLT_KT, PROG_P1>, g, dim3(256), 0, s, a, st, nelem);
  else if (prog == PROG_P3) launch_timed(kind, pointwise_kernel<MOLT_KT, PROG_P3>, g, dim3(256), 0, s, a, st, nelem);
  else if (prog == PROG_P1V) launch_timed(kind, pointwise_kernel<MOLT_KT, PROG_P1V>, g, dim3(256), 0, s, a, st, nelem);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t MOLT_KFN(launch_copy)(void* dst, const void* src, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((copy_kernel<MOLT_KT>), grid_1d(n), dim3(256), 0, s, (MOLT_KT*)dst, (const MOLT_KT*)src, n);
  return hipGetLastError();
}

hipError_t MOLT_KFN(launch_finalize)(void* u, const void* base, const void* W, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((finalize_kernel<MOLT_KT>), grid_1d(n), dim3(256), 0, s, (MOLT_KT*)u, (const MOLT_KT*)base,
                     (const MOLT_KT*)W, n);
  return hipGetLastError();
}

hipError_t MOLT_KFN(launch_vch_react)(const PassArgs& a, DevState* st, size_t n, hipStream_t s) {
  dim3 g = grid_1d(n);
  launch_timed(prof_kind<MOLT_KT>(KF_POINTWISE * 8 + PROG_P1V), vch_react_kernel<MOLT_KT>, g, dim3(256), 0, s, a, st,
               n);
  return hipGetLastError();
}

hipError_t MOLT_KFN(launch_diag_vch)(const void* u, int nx, int ny, int bc, double hx, double hy, double eps,
                                     double* partials, DevState* st, hipStream_t s) {
  const int nb = diag_blocks((size_t)nx * ny);
  hipLaunchKernelGGL((diag_vch_kernel<MOLT_KT>), dim3(nb), dim3(256), 0, s, (const MOLT_KT*)u, nx, ny, bc, hx, hy, eps,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((diag_vch_final_kernel<MOLT_KT>), dim3(1), dim3(256), 0, s, (const double*)partials, nb, hx * hy,
                     st);
  return hipGetLastError();
}

// out = x + c (y - x)
template <typename T>
__global__ void __launch_bounds__(256) lerp_kernel(T* out, const T* x, const T* y, double c, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = x[i] + (T)c * (y[i] - x[i]);
}

hipError_t MOLT_KFN(launch_lerp)(void* out, const void* x, const void* y, double c, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((lerp_kernel<MOLT_KT>), grid_1d(n), dim3(256), 0, s, (MOLT_KT*)out, (const MOLT_KT*)x,
                     (const MOLT_KT*)y, c, n);
  return hipGetLastError();
}

// x += c0 on the first n values, x += c1 on the next n (nc = 2)
template <typename T>
__global__ void __launch_bounds__(256) addc_kernel(T* x, double c0, double c1, size_t n, int nc) {
  const size_t tot = n * (size_t)nc;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (size_t)gridDim.x * blockDim.x)
    x[i] += (T)(i < n ? c0 : c1);
}

hipError_t MOLT_KFN(launch_addc)(void* x, double c0, double c1, size_t n, int nc, hipStream_t s) {
  hipLaunchKernelGGL((addc_kernel<MOLT_KT>), grid_1d(n * (size_t)nc), dim3(256), 0, s, (MOLT_KT*)x, c0, c1, n, nc);
  return hipGetLastError();
}

// max |a - b| -> out[0] (partials: diag_blocks(n) doubles)
hipError_t MOLT_KFN(launch_maxdiff)(const void* a, const void* b, size_t n, double* partials, double* out,
                                    hipStream_t s) {
  const int nb = diag_blocks(n);
  hipLaunchKernelGGL((maxdiff_kernel<MOLT_KT>), dim3(nb), dim3(256), 0, s, (const MOLT_KT*)a, (const MOLT_KT*)b, n,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((maxdiff_final_kernel<MOLT_KT>), dim3(1), dim3(64), 0, s, (const double*)partials, nb, out);
  return hipGetLastError();
}

hipError_t MOLT_KFN(launch_diag)(const void* u, int nx, int ny, int bc, double hx, double hy, double eps,
                                 double* partials, DevState* st, hipStream_t s) {
  const int nb = diag_blocks((size_t)nx * ny);
  hipLaunchKernelGGL((diag_kernel<MOLT_KT>), dim3(nb), dim3(256), 0, s, (const MOLT_KT*)u, nx, ny, bc, hx, hy, eps,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((diag_final_kernel<MOLT_KT>), dim3(1), dim3(256), 0, s, (const double*)partials, nb, hx * hy, st);
  return hipGetLastError();
}
#endif  // MOLT_PART_Y

}  // namespace molt
