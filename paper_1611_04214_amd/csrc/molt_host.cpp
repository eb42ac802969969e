// molt_host.cpp -- host side of libmolt: argument checks, stepper parameters,
// quadrature weights, workspace layout, the time-step driver and the C-ABI.
#include <math.h>
#include <string.h>

#include <atomic>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "molt.h"
#include "molt_internal.h"

namespace molt {
// single-problem kernels, one translation unit per precision and pass direction
#define MOLT_KERN_DECL(sfx)                                                                                     \
  hipError_t launch_xpass_##sfx(int prog, const LineCoef& c, const PassArgs& a, DevState* st, int nlines,     \
                                double* rpart, hipStream_t s);                                                 \
  hipError_t launch_ypass_##sfx(int prog, const LineCoef& c, const PassArgs& a, DevState* st, int nx,         \
                                int batch, void* tot, void* jln, bool deferred, hipStream_t s);                \
  hipError_t launch_pointwise_##sfx(int prog, const PassArgs& a, DevState* st, size_t nelem, hipStream_t s);  \
  hipError_t launch_copy_##sfx(void* dst, const void* src, size_t n, hipStream_t s);                          \
  hipError_t launch_finalize_##sfx(void* u, const void* base, const void* W, size_t n, hipStream_t s);        \
  hipError_t launch_diag_##sfx(const void* u, int nx, int ny, int bc, double hx, double hy, double eps,       \
                               double* partials, DevState* st, hipStream_t s);                                \
  hipError_t launch_diag_vch_##sfx(const void* u, int nx, int ny, int bc, double hx, double hy, double eps,   \
                                   double* partials, DevState* st, hipStream_t s);                             \
  hipError_t launch_vch_react_##sfx(const PassArgs& a, DevState* st, size_t n, hipStream_t s);                  \
  hipError_t launch_maxdiff_##sfx(const void* a, const void* b, size_t n, double* partials, double* out,      \
                                  hipStream_t s);                                                              \
  hipError_t launch_lerp_##sfx(void* out, const void* x, const void* y, double c, size_t n, hipStream_t s); \
  hipError_t launch_addc_##sfx(void* x, double c0, double c1, size_t n, int nc, hipStream_t s);
MOLT_KERN_DECL(f32)
MOLT_KERN_DECL(f64)
#undef MOLT_KERN_DECL
#define MOLT_PREC(call) (prec == MOLT_F64 ? call##_f64 : call##_f32)
hipError_t launch_xpass(int prec, int prog, const LineCoef& c, const PassArgs& a, DevState* st, int nlines,
                        double* rpart, hipStream_t s) {
  return MOLT_PREC(launch_xpass)(prog, c, a, st, nlines, rpart, s);
}
hipError_t launch_ypass(int prec, int prog, const LineCoef& c, const PassArgs& a, DevState* st, int nx, int batch,
                        void* tot, void* jln, bool deferred, hipStream_t s) {
  return MOLT_PREC(launch_ypass)(prog, c, a, st, nx, batch, tot, jln, deferred, s);
}
static hipError_t launch_pointwise(int prec, int prog, const PassArgs& a, DevState* st, size_t nelem, hipStream_t s) {
  return MOLT_PREC(launch_pointwise)(prog, a, st, nelem, s);
}
static hipError_t launch_copy(int prec, void* dst, const void* src, size_t n, hipStream_t s) {
  return MOLT_PREC(launch_copy)(dst, src, n, s);
}
static hipError_t launch_finalize(int prec, void* u, const void* base, const void* W, size_t n, hipStream_t s) {
  return MOLT_PREC(launch_finalize)(u, base, W, n, s);
}
static hipError_t launch_diag(int prec, const void* u, int nx, int ny, int bc, double hx, double hy, double eps,
                              double* partials, DevState* st, hipStream_t s) {
  return MOLT_PREC(launch_diag)(u, nx, ny, bc, hx, hy, eps, partials, st, s);
}
static hipError_t launch_diag_vch(int prec, const void* u, int nx, int ny, int bc, double hx, double hy, double eps,
                                  double* partials, DevState* st, hipStream_t s) {
  return MOLT_PREC(launch_diag_vch)(u, nx, ny, bc, hx, hy, eps, partials, st, s);
}
static hipError_t launch_vch_react(int prec, const PassArgs& a, DevState* st, size_t n, hipStream_t s) {
  return MOLT_PREC(launch_vch_react)(a, st, n, s);
}
static hipError_t launch_maxdiff(int prec, const void* a, const void* b, size_t n, double* partials, double* out,
                                 hipStream_t s) {
  return MOLT_PREC(launch_maxdiff)(a, b, n, partials, out, s);
}
static hipError_t launch_lerp(int prec, void* out, const void* x, const void* y, double c, size_t n, hipStream_t s) {
  return MOLT_PREC(launch_lerp)(out, x, y, c, n, s);
}
static hipError_t launch_addc(int prec, void* x, double c0, double c1, size_t n, int nc, hipStream_t s) {
  return MOLT_PREC(launch_addc)(x, c0, c1, n, nc, s);
}
#undef MOLT_PREC
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
hipError_t launch_widen(void* dst64, const void* src32, size_t n, hipStream_t s);
hipError_t launch_iterate64(void* v64, const void* base32, const void* W32, const DevState* st, size_t n,
                            hipStream_t s);
hipError_t launch_close_pending(const double* rpart, DevState* st, hipStream_t s);

hipError_t launch_state_init(DevState* st, double tol, int max_iter, int fixed, hipStream_t s);
size_t ypass_tot_elems(int prec, int n, int nx, int batch);
int diag_blocks(size_t n);
int xpass_max_n(int prec);

int xpass_pick_k(int n, int prec);
int xpass_pick_k256(int n, int prec);
int xpass_tl(int n, int K);
void ypass_shape(int prec, int n, int* nth, int* nseg);
// batched kernels, one translation unit per precision
#define MOLT_BATCH_DECL(sfx)                                                                                    \
  hipError_t launch_batch_y_##sfx(int K, int M, bool per, int pass, const SlotDesc* sd,                        \
                                  const SlotCtl* ctl, const BlkMap* map, int nblk, hipStream_t s);             \
  hipError_t launch_batch_comb_##sfx(int pass, const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* map,      \
                                     int nblk, hipStream_t s);                                                 \
  hipError_t launch_batch_x_##sfx(int K, int M, bool per, int pass, const SlotDesc* sd, const SlotCtl* ctl,    \
                                  const BlkMap* map, int nblk, hipStream_t s);                                 \
  hipError_t launch_batch_tail_##sfx(const SlotDesc* sd, SlotCtl* ctl, const BlkMap* slots, int nslots,        \
                                     const BlkMap* pmap, int npblk, bool close_only, bool hybrid,              \
                                     hipStream_t s);                                                           \
  hipError_t launch_batch_react_##sfx(const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* pmap, int npblk,   \
                                      hipStream_t s);                                                          \
  hipError_t launch_batch_init_##sfx(const SlotDesc* sd, SlotCtl* ctl, int nslots, hipStream_t s);             \
  hipError_t launch_batch_count_##sfx(const SlotCtl* ctl, int nslots, int* out, hipStream_t s);
MOLT_BATCH_DECL(f32)
MOLT_BATCH_DECL(f64)
#undef MOLT_BATCH_DECL
hipError_t launch_batch_widen(const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* pmap, int npblk, hipStream_t s);
int ypass_pick_k(int n, int prec);
int ypass_max_segments(int n);
int xpass_min_k(int n, int prec);
int tune_class(int n);
bool tune_valid(int prec, int cls, int kx, int ky);
void tune_get(int prec, int cls, int* kx, int* ky);
void tune_set(int prec, int cls, int kx, int ky);

enum { PROG_SWEEP = 0, PROG_RHS = 1, PROG_P1 = 2, PROG_P2 = 3, PROG_P3 = 4, PROG_P4 = 5, PROG_P1V = 6, PROG_P2V = 7,
       PROG_P2F = 8, PROG_P4F = 9, PROG_RHSW = 10, PROG_P4R = 11 };

// --------------------------------------------------------------------------
// errors
// --------------------------------------------------------------------------
static thread_local std::string g_err;

static int32_t fail(int32_t code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(MOLT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// --------------------------------------------------------------------------
// per-kernel HIP-event profiler (process-wide; meant for one profiling thread)
// --------------------------------------------------------------------------
bool g_prof_on = false;
static int g_batch_ticks = 8;                     // batched solve: ticks between host checks
static int g_batch_graph = 1;                     // batched solve: replay the ticks as a HIP graph
static int g_batch_lean = 16;                     // batched solve: lean ticks with at most this many instances
namespace {
struct PendingEv {
  int kind;
  hipEvent_t b, e;
};
std::mutex g_prof_mu;
std::vector<hipEvent_t> g_ev_pool;
std::vector<PendingEv> g_pending;
hipEvent_t g_open[kProfKinds];
double g_prof_ms[kProfKinds];
long long g_prof_n[kProfKinds];

hipEvent_t ev_get() {
  if (!g_ev_pool.empty()) {
    hipEvent_t e = g_ev_pool.back();
    g_ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

static int g_prof_only = -1;  // time only this kind (-1: every kind)

void prof_begin(int kind, hipStream_t s) {
  if (g_prof_only >= 0 && kind != g_prof_only) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = ev_get();
  if (e) (void)hipEventRecord(e, s);
  g_open[kind] = e;
}

void prof_end(int kind, hipStream_t s) {
  if (g_prof_only >= 0 && kind != g_prof_only) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = ev_get();
  if (e) (void)hipEventRecord(e, s);
  if (g_open[kind] && e) g_pending.push_back({kind, g_open[kind], e});
  g_open[kind] = nullptr;
}

void prof_pair(int kind, hipEvent_t* b, hipEvent_t* e) {
  *b = *e = nullptr;
  if (g_prof_only >= 0 && kind != g_prof_only) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t x = ev_get(), y = ev_get();
  if (x && y) {
    g_pending.push_back({kind, x, y});
    *b = x;
    *e = y;
    return;
  }
  if (x) g_ev_pool.push_back(x);
  if (y) g_ev_pool.push_back(y);
}

// accumulate every recorded pair (the caller has synchronized the stream)
static void prof_drain() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (const PendingEv& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.e) == hipSuccess && hipEventElapsedTime(&ms, p.b, p.e) == hipSuccess) {
      g_prof_ms[p.kind] += ms;
      g_prof_n[p.kind] += 1;
    }
    g_ev_pool.push_back(p.b);
    g_ev_pool.push_back(p.e);
  }
  g_pending.clear();
}

// --------------------------------------------------------------------------
// quadrature weights (Sec. 3.2): the local integral over one cell with kernel
// alpha*exp(-alpha|x_j - x'|) of the degree-M Lagrange interpolant on the M+1
// nodes centred at j.  With s = |x_j - x'|/h in [0,1]:
//   J^L weight of node j+t_i = sum_p c_p mu_p,  l_i(-s) = sum_p c_p s^p,
//   mu_p(nu) = nu * int_0^1 exp(-nu s) s^p ds,
// and J^R the same with l_i(+s).  mu_p in long double: power series for
// nu <= M+1, the upward recurrence mu_p = (p/nu) mu_{p-1} - e^{-nu} (stable for
// p < nu) above.
// --------------------------------------------------------------------------
static void moments(int M, long double nu, long double* mu) {
  if (nu > (long double)(M + 1)) {
    const long double e = expl(-nu);
    mu[0] = -expm1l(-nu);
    for (int p = 1; p <= M; ++p) mu[p] = ((long double)p / nu) * mu[p - 1] - e;
  } else {
    for (int p = 0; p <= M; ++p) {
      long double sum = 0.0L, term = 1.0L;  // (-nu)^q / q!
      for (int q = 0; q < 400; ++q) {
        const long double add = term / (long double)(p + q + 1);
        sum += add;
        if (q > 2 && fabsl(add) < 1e-24L * fabsl(sum)) break;
        term *= -nu / (long double)(q + 1);
      }
      mu[p] = nu * sum;
    }
  }
}

// coefficients in s of the Lagrange basis polynomial i on nodes t_k = k - M/2,
// evaluated at sign*s
static void lagrange_in_s(int M, int i, int sign, long double* coef) {
  for (int p = 0; p <= M; ++p) coef[p] = 0.0L;
  coef[0] = 1.0L;
  int deg = 0;
  const long double ti = (long double)(i - M / 2);
  for (int k = 0; k <= M; ++k) {
    if (k == i) continue;
    const long double tk = (long double)(k - M / 2);
    const long double den = ti - tk;
    // multiply by (sign*s - tk)/den
    long double nw[kMaxM + 2];
    for (int p = 0; p <= deg + 1; ++p) nw[p] = 0.0L;
    for (int p = 0; p <= deg; ++p) {
      nw[p] += -tk * coef[p] / den;
      nw[p + 1] += (long double)sign * coef[p] / den;
    }
    ++deg;
    for (int p = 0; p <= deg; ++p) coef[p] = nw[p];
  }
}

// Lagrange basis i on nodes 0..M at x
static long double lagrange_at(int M, int i, long double x) {
  long double p = 1.0L;
  for (int k = 0; k <= M; ++k)
    if (k != i) p *= (x - (long double)k) / (long double)(i - k);
  return p;
}

static double spacing(int bc, int n, double a, double b) {
  return bc == MOLT_BC_PERIODIC ? (b - a) / n : (b - a) / (n - 1);
}

static LineCoef make_line(int n, int bc, int M, double alpha, double h) {
  LineCoef c;
  memset(&c, 0, sizeof(c));
  c.n = n;
  c.N = bc == MOLT_BC_PERIODIC ? n : n - 1;
  c.bc = bc;
  c.M = M;
  const long double nu = (long double)alpha * (long double)h;
  c.nu = (double)nu;
  c.d = (double)expl(-nu);
  c.mu = (double)expl(-nu * (long double)c.N);
  long double mu[kMaxM + 1], cf[kMaxM + 2];
  moments(M, nu, mu);
  for (int i = 0; i <= M; ++i) {
    long double sl = 0.0L, sr = 0.0L;
    lagrange_in_s(M, i, -1, cf);
    for (int p = 0; p <= M; ++p) sl += cf[p] * mu[p];
    lagrange_in_s(M, i, +1, cf);
    for (int p = 0; p <= M; ++p) sr += cf[p] * mu[p];
    c.wl[i] = (double)sl;
    c.wr[i] = (double)sr;
  }
  for (int g = 1; g <= M / 2; ++g)
    for (int i = 0; i <= M; ++i) {
      c.ghostL[g - 1][i] = (double)lagrange_at(M, i, -(long double)g);
      c.ghostR[g - 1][i] = (double)lagrange_at(M, i, (long double)(M + g));
    }
  return c;
}

// --------------------------------------------------------------------------
// stepper parameters (Sec. 3.1, 4.1): (I - sigma a Lap + a eps^2 Lap^2) =
// (I - s1 Lap)(I - s2 Lap), a = beta dt; sigma = sigma0 when the roots are real
// (factorization), otherwise the square is completed with sigma = 2 eps/sqrt(a)
// and s1 = s2 = eps sqrt(a).
// --------------------------------------------------------------------------
struct StepParams {
  double a, s1, s2, sigma;
};

static StepParams step_params(double eps, double dt, double beta, double sigma0) {
  StepParams p;
  p.a = beta * dt;
  const double half = 0.5 * sigma0 * p.a, prod = p.a * eps * eps;
  if (half * half >= prod) {
    p.sigma = sigma0;
    p.s1 = half + sqrt(half * half - prod);
    p.s2 = prod / p.s1;
  } else {
    p.s1 = p.s2 = sqrt(prod);
    p.sigma = 2.0 * eps / sqrt(p.a);
  }
  return p;
}

// --------------------------------------------------------------------------
// validation and workspace layout
// --------------------------------------------------------------------------
static int32_t check_grid(const molt_grid* g, int prec) {
  if (!g) return fail(MOLT_EINVAL, "grid is NULL");
  if (g->order_M != 2 && g->order_M != 4 && g->order_M != 6) return fail(MOLT_EINVAL, "order_M must be 2, 4 or 6");
  if (g->bc != MOLT_BC_PERIODIC && g->bc != MOLT_BC_NEUMANN && g->bc != MOLT_BC_DIRICHLET)
    return fail(MOLT_EINVAL, "unknown boundary condition");
  if (prec != MOLT_F64 && prec != MOLT_F32) return fail(MOLT_EINVAL, "unknown precision");
  if (g->nx < g->order_M + 1) return fail(MOLT_EINVAL, "nx must be at least M+1");
  if (g->ny != 1 && g->ny < g->order_M + 1) return fail(MOLT_EINVAL, "ny must be 1 or at least M+1");
  if (!(g->x1 > g->x0)) return fail(MOLT_EINVAL, "x1 must exceed x0");
  if (g->ny > 1 && !(g->y1 > g->y0)) return fail(MOLT_EINVAL, "y1 must exceed y0");
  if (g->nx > xpass_max_n(prec) || g->ny > xpass_max_n(prec))
    return fail(MOLT_EUNSUPPORTED, "lines longer than 8192 (FP32) / 4096 (FP64) nodes");
  return MOLT_OK;
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of one problem.  An FP32 problem also holds an FP64 shadow: the
// right-hand side sweeps R = A1^{-1} A2^{-1} rhs and the first (full-form)
// fixed-point iteration of every step run in FP64 on it (fld64, tot64, jln64,
// and FP64 copies of the step's inputs in64), and only the increments of the
// later iterations run in FP32.  The splitting's fixed point amplifies an
// error in its data by (I - T)^{-1}, whose largest entries (modes that are
// high in both directions, small alpha*h) are ~1/(4 lambda^2): FP32 rounding
// of R or of the first increment, at the ulp of u, would be amplified to a
// persistent drift instead of a 1e-8 increment.
struct Layout {
  size_t fld[F_COUNT];
  size_t tot, jln, state, partials, rpart;
  bool hybrid;               // FP32 problem with its FP64 shadow
  size_t fld64[F_COUNT];     // FP64 shadow fields (hybrid only)
  size_t tot64, jln64;       // FP64 y-pass scratch
  size_t in64[3];            // FP64 copies of u^n, u^{n-1}, u^{n-2}
  size_t total;
};

static int ncomp_of(const molt_ch_params* p) { return p->model == MOLT_MODEL_VCH ? 2 : 1; }

static bool field_used(int i, int ncomp, bool bdf3) {
  if (i == F_E || i == F_LIN) return ncomp == 2;
  if (i == F_HIST2 || i == F_STAGE) return bdf3;
  return true;
}

static Layout ch_layout(const molt_grid* g, int prec, int ncomp, bool bdf3 = false) {
  Layout L;
  memset(&L, 0, sizeof(L));
  const size_t esz = prec == MOLT_F64 ? 8 : 4;
  const size_t n = (size_t)g->nx * g->ny;
  size_t off = 0;
  for (int i = 0; i < F_COUNT; ++i) {
    L.fld[i] = off;
    off += field_used(i, ncomp, bdf3) ? al256(n * ncomp * esz) : 0;
  }
  L.tot = off;
  off += al256(g->ny > 1 ? ypass_tot_elems(prec, g->ny, g->nx, ncomp) * esz : 0);
  L.jln = off;
  off += al256((size_t)2 * g->nx * ncomp * esz);
  L.state = off;
  off += al256(sizeof(DevState));
  L.partials = off;  // mass / energy partials: up to three per diagnostic block
  off += al256((size_t)3 * diag_blocks(n) * sizeof(double));
  L.rpart = off;  // one residual slot per x-pass block (at most one block per row)
  off += al256((size_t)g->ny * ncomp * sizeof(double));
  L.hybrid = prec == MOLT_F32;
  if (L.hybrid) {
    for (int i = 0; i < F_COUNT; ++i) {
      L.fld64[i] = off;
      off += field_used(i, ncomp, bdf3) ? al256(n * ncomp * 8) : 0;
    }
    L.tot64 = off;
    off += al256(g->ny > 1 ? ypass_tot_elems(MOLT_F64, g->ny, g->nx, ncomp) * 8 : 0);
    L.jln64 = off;
    off += al256((size_t)2 * g->nx * ncomp * 8);
    for (int i = 0; i < 3; ++i) {
      L.in64[i] = off;
      off += (i < 2 || bdf3) ? al256(n * ncomp * 8) : 0;
    }
  }
  L.total = off;
  return L;
}

// --------------------------------------------------------------------------
// one step
// --------------------------------------------------------------------------
// The line coefficients and launch geometry of one step.
struct StepGeo {
  int nx, ny, nc, xl;  // xl: x-lines (ny rows per component)
  size_t n;            // nodes per component
  bool two_d, vch;
  LineCoef cx1, cx2, cy1, cy2;
};

// The corrections the x-pass after a deferred y-pass (program with nf swept
// fields along the lines c) adds to what it reads from it (see YCorr)
static YCorr make_ycorr(int prec, const LineCoef& c, int nx, int nf, const void* tot) {
  YCorr y;
  int nth = 0, nseg = 0;
  ypass_shape(prec, c.n, &nth, &nseg);
  y.seeds = tot;
  y.nf = nf;
  y.nseg = nseg;
  y.S = kRG * ypass_pick_k(c.n, prec);
  y.ny = c.n;
  y.nx = nx;
  y.nu = c.nu;
  return y;
}

// R = A1^{-1} A2^{-1} rhs, A_i^{-1} = Lx_i^{-1} Ly_i^{-1} (Sec. 5.1, first term
// of eq. CH_BE_2D_3), with rhs of the stepper (eq. CH_BE; eqs. BDF2, BDF3) from
// in0..in2 = u^n, u^{n-1}, u^{n-2}; A1, B1 are scratch fields of the precision
// (rhs_prog: PROG_RHS, or PROG_RHSW for FP64 kernels reading FP32 fields)
static int32_t enqueue_rhs(int prec, const StepGeo& G, const PassArgs& rhs_args, void* const* F, void* tot, void* jln,
                           DevState* st, hipStream_t s, int rhs_prog = PROG_RHS) {
  PassArgs a = rhs_args;
  if (G.two_d) {
    a.out[0] = F[F_A1];
    HIPCHK(launch_ypass(prec, rhs_prog, G.cy2, a, st, G.nx, G.nc, tot, jln, true, s));
    a.in[0] = F[F_A1];
    a.out[0] = F[F_B1];
    a.corr = make_ycorr(prec, G.cy2, G.nx, 1, tot);
    HIPCHK(launch_xpass(prec, PROG_SWEEP, G.cx2, a, nullptr, G.xl, nullptr, s));
    a.corr.seeds = nullptr;
    a.in[0] = F[F_B1];
    a.out[0] = F[F_A1];
    HIPCHK(launch_ypass(prec, PROG_SWEEP, G.cy1, a, st, G.nx, G.nc, tot, jln, true, s));
    a.in[0] = F[F_A1];
    a.out[0] = F[F_R];
    a.corr = make_ycorr(prec, G.cy1, G.nx, 1, tot);
    HIPCHK(launch_xpass(prec, PROG_SWEEP, G.cx1, a, nullptr, G.xl, nullptr, s));
  } else {
    a.out[0] = F[F_B1];
    HIPCHK(launch_xpass(prec, rhs_prog, G.cx2, a, nullptr, G.xl, nullptr, s));
    a.in[0] = F[F_B1];
    a.out[0] = F[F_R];
    HIPCHK(launch_xpass(prec, PROG_SWEEP, G.cx1, a, nullptr, G.xl, nullptr, s));
  }
  return MOLT_OK;
}

// One fixed-point iteration (Sec. 5.1, eqs. CH_BE_2D_3, CH_2D_Doperator1/2) as
// the four passes P1..P4 on the fields F of the precision; mode 0 the full form
// from the iterate `base`, mode 1 the increment form (base + W the iterate,
// DL the last increment).  P4 writes DL, W and the residual partials; the
// close (residual, count, stop) follows it, or with defer_close is left to
// the next iteration's P1 y-pass or an explicit close.  P1 (2D) always closes
// a pending previous iteration first.  F32 (an FP64 full-form iteration of an
// FP32 step): P4 writes the re-based FP32 iterate -- base fl32(v), running sum
// v - fl32(v), increment -- into those fields instead of its FP64 outputs.
static int32_t enqueue_iteration(int prec, const StepGeo& G, const StepParams& sp, const double* ush, int mode,
                                 const void* base, void* const* F, void* tot, void* jln, DevState* st, double* rpart,
                                 bool defer_close, hipStream_t s, void* const* F32) {
  PassArgs q;
  memset(&q, 0, sizeof(q));
  q.sigma = sp.sigma;
  q.kappa = sp.a / sp.s1;
  q.mode = mode;
  q.ushift[0] = ush[0];
  q.ushift[1] = ush[1];
  // P1 (y, alpha1): a1 = Y1 e, b1 = Y1 lin (vector model: e, lin from the
  // pointwise reaction pass, then both components swept as a batch)
  q.in[0] = base;
  q.in[1] = F[F_W];
  q.in[2] = F[F_DL];
  if (G.vch) {
    q.out[0] = F[F_E];
    q.out[1] = F[F_LIN];
    HIPCHK(launch_vch_react(prec, q, st, G.n, s));
    q.in[0] = F[F_E];
    q.in[1] = F[F_LIN];
    q.in[2] = nullptr;
  }
  q.out[0] = F[F_A1];
  q.out[1] = F[F_B1];
  const int p1 = G.vch ? PROG_P1V : PROG_P1;
  if (G.two_d) {
    q.close_part = rpart;
    HIPCHK(launch_ypass(prec, p1, G.cy1, q, st, G.nx, G.nc, tot, jln, true, s));
    q.close_part = nullptr;
    q.corr = make_ycorr(prec, G.cy1, G.nx, 2, tot);
  } else {
    HIPCHK(launch_pointwise(prec, p1, q, st, G.n * G.nc, s));
  }
  // P2 (x, alpha1): C, q
  q.in[0] = F[F_A1];
  q.in[1] = F[F_B1];
  if (G.vch) {
    q.in[2] = F[F_E];
    q.in[3] = F[F_LIN];
    q.in[4] = nullptr;
  } else {
    q.in[2] = base;
    q.in[3] = F[F_W];
    q.in[4] = F[F_DL];
  }
  q.out[0] = F[F_C];
  q.out[1] = F[F_Q];
  // (FP64 full form: the programs without the increment-form inputs)
  const bool full64 = prec == MOLT_F64 && mode == 0;
  HIPCHK(launch_xpass(prec, G.vch ? PROG_P2V : (full64 ? PROG_P2F : PROG_P2), G.cx1, q, st, G.xl, nullptr, s));
  q.corr.seeds = nullptr;
  // P3 (y, alpha2): m, n
  q.in[0] = F[F_C];
  q.in[1] = F[F_Q];
  q.in[2] = q.in[3] = q.in[4] = nullptr;
  q.out[0] = F[F_M];
  q.out[1] = F[F_N];
  if (G.two_d) {
    HIPCHK(launch_ypass(prec, PROG_P3, G.cy2, q, st, G.nx, G.nc, tot, jln, true, s));
    q.corr = make_ycorr(prec, G.cy2, G.nx, 2, tot);
  } else {
    HIPCHK(launch_pointwise(prec, PROG_P3, q, st, G.n * G.nc, s));
  }
  // P4 (x, alpha2): increment and running sum, residual
  q.in[0] = F[F_M];
  q.in[1] = F[F_N];
  q.in[2] = mode ? F[F_DL] : F[F_R];
  q.in[3] = F[F_W];
  q.out[0] = F[F_DL];
  q.out[1] = F[F_W];
  q.defer_close = defer_close && G.two_d ? 1 : 0;
  int p4 = full64 ? PROG_P4F : PROG_P4;
  if (full64 && F32 != nullptr) {
    p4 = PROG_P4R;
    q.in[3] = base;  // (read late: after the program's three raw fields)
    q.out[0] = F32[F_DL];
    q.out[1] = F32[F_W];
    q.out[2] = F32[F_R];
  }
  HIPCHK(launch_xpass(prec, p4, G.cx2, q, st, G.xl, rpart, s));
  return MOLT_OK;
}

#define MOLT_RC(expr)                     \
  do {                                    \
    const int32_t rc_ = (expr);           \
    if (rc_ != MOLT_OK) return rc_;       \
  } while (0)

// --------------------------------------------------------------------------
// Runs of increment-form iterations replayed as executable graphs.  Every
// increment iteration of a step launches the same kernels with the same
// arguments (what changes lives in the device state), so a run of kIterRun of
// them is captured once -- on a private stream of the library, so that the
// caller's stream (the null stream included) need not support capture -- and
// then launched on the caller's stream, one launch in place of ~7 per
// iteration.  The graphs are cached by everything their kernels are given:
// device, precision, geometry and line coefficients, step parameters, the
// workspace's field pointers and the line-block shapes in force.
// --------------------------------------------------------------------------
constexpr int kIterRun = 4;
constexpr int kIterGraphs = 8;  // cached graphs (least recently used replaced)

struct IterKey {
  int dev, prec, mode;
  int kx, ky;
  StepGeo G;
  double sigma, kappa, s1, ush[2];
  const void* base;
  void* F[F_COUNT];
  void* tot;
  void* jln;
  DevState* st;
  double* rpart;
};

struct IterGraph {
  IterKey key;
  hipGraphExec_t exec;
  unsigned long long used;
};

static std::mutex g_graph_mu;
static std::vector<IterGraph> g_iter_graphs;
static unsigned long long g_graph_clock = 0;
static std::atomic<bool> g_iter_graph_on{true};
static std::map<int, hipStream_t> g_capture_streams;

static hipStream_t capture_stream(int dev) {
  auto it = g_capture_streams.find(dev);
  if (it != g_capture_streams.end()) return it->second;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
  g_capture_streams[dev] = cs;
  return cs;
}

// forward declaration (defined below)
static int32_t enqueue_iteration(int prec, const StepGeo& G, const StepParams& sp, const double* ush, int mode,
                                 const void* base, void* const* F, void* tot, void* jln, DevState* st, double* rpart,
                                 bool defer_close, hipStream_t s, void* const* F32 = nullptr);

// the executable graph of kIterRun increment iterations for this key, captured
// on first use; nullptr when graphs are off or the capture failed (the caller
// then launches the kernels itself)
static hipGraphExec_t iteration_graph(int prec, const StepGeo& G, const StepParams& sp, const double* ush,
                                      const void* base, void* const* F, void* tot, void* jln, DevState* st,
                                      double* rpart) {
  if (!g_iter_graph_on || g_prof_on) return nullptr;
  IterKey k;
  memset(&k, 0, sizeof(k));
  if (hipGetDevice(&k.dev) != hipSuccess) return nullptr;
  k.prec = prec;
  k.mode = 1;
  k.kx = xpass_pick_k(G.nx, prec);
  k.ky = G.two_d ? ypass_pick_k(G.ny, prec) : 0;
  k.G = G;
  k.sigma = sp.sigma;
  k.kappa = sp.a;
  k.s1 = sp.s1;
  k.ush[0] = ush[0];
  k.ush[1] = ush[1];
  k.base = base;
  for (int i = 0; i < F_COUNT; ++i) k.F[i] = F[i];
  k.tot = tot;
  k.jln = jln;
  k.st = st;
  k.rpart = rpart;
  std::lock_guard<std::mutex> lock(g_graph_mu);
  for (IterGraph& e : g_iter_graphs)
    if (memcmp(&e.key, &k, sizeof(k)) == 0) {
      e.used = ++g_graph_clock;
      return e.exec;
    }
  hipStream_t cs = capture_stream(k.dev);
  if (cs == nullptr) return nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) return nullptr;
  int32_t rc = MOLT_OK;
  for (int i = 0; i < kIterRun && rc == MOLT_OK; ++i)
    rc = enqueue_iteration(prec, G, sp, ush, 1, base, F, tot, jln, st, rpart, G.two_d, cs);
  const hipError_t e = hipStreamEndCapture(cs, &graph);
  if (rc == MOLT_OK && e == hipSuccess && graph != nullptr &&
      hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
    exec = nullptr;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipGetLastError();
  if (exec == nullptr) return nullptr;
  if ((int)g_iter_graphs.size() >= kIterGraphs) {
    size_t lru = 0;
    for (size_t i = 1; i < g_iter_graphs.size(); ++i)
      if (g_iter_graphs[i].used < g_iter_graphs[lru].used) lru = i;
    // launches of the evicted graph may still be queued
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(g_iter_graphs[lru].exec);
    g_iter_graphs.erase(g_iter_graphs.begin() + lru);
  }
  g_iter_graphs.push_back(IterGraph{k, exec, ++g_graph_clock});
  return exec;
}

// host copy of the device state, read back after each batch of iterations
// (pinned, so that the read is one direct copy)
static DevState* state_readback() {
  static thread_local DevState* pin = nullptr;
  if (pin == nullptr && hipHostMalloc((void**)&pin, sizeof(DevState), hipHostMallocPortable) != hipSuccess)
    pin = nullptr;
  return pin;
}

// iteration count of the last step run in each workspace: the batch hint of
// the next ch_step call on it (callers that step one call at a time)
static std::mutex g_hint_mu;
static std::map<const void*, int> g_last_iters;

static int workspace_hint(const void* w) {
  std::lock_guard<std::mutex> lock(g_hint_mu);
  auto it = g_last_iters.find(w);
  return it == g_last_iters.end() ? 0 : it->second;
}

static void workspace_hint_set(const void* w, int iters) {
  std::lock_guard<std::mutex> lock(g_hint_mu);
  if (g_last_iters.size() >= 256 && g_last_iters.find(w) == g_last_iters.end()) g_last_iters.clear();
  g_last_iters[w] = iters;
}

// omega: BDF2 step ratio dt_n / dt_{n-1} (1: constant steps, eq. BDF2; otherwise the variable-step form)
// d_u_prev2 (with bdf2): a BDF3 step (eq. BDF3) from u^n, u^{n-1}, u^{n-2}
static int32_t step_impl(const molt_grid* g, const molt_ch_params* p, void* d_u, void* d_u_prev, bool bdf2,
                         void* d_work, size_t work_bytes, molt_step_info* info, hipStream_t s, int iter_hint,
                         double omega = 1.0, void* d_u_prev2 = nullptr) {
  const int prec = p->precision;
  const int nc = ncomp_of(p);
  const bool vch = nc == 2;
  const bool bdf3 = bdf2 && d_u_prev2 != nullptr;
  const Layout L = ch_layout(g, prec, nc, p->stepper == MOLT_BDF3);
  if (!d_work || work_bytes < L.total) return fail(MOLT_EWORKSPACE, "workspace smaller than ch_workspace_bytes()");
  char* w = (char*)d_work;
  void* F[F_COUNT];
  void* F64[F_COUNT];
  for (int i = 0; i < F_COUNT; ++i) {
    F[i] = w + L.fld[i];
    F64[i] = L.hybrid ? w + L.fld64[i] : nullptr;
  }
  void* tot = w + L.tot;
  void* jln = w + L.jln;
  DevState* st = (DevState*)(w + L.state);
  double* partials = (double*)(w + L.partials);
  double* rpart = (double*)(w + L.rpart);

  StepGeo G;
  memset(&G, 0, sizeof(G));  // (graph keys compare it byte for byte)
  G.nx = g->nx;
  G.ny = g->ny;
  G.nc = nc;
  G.vch = vch;
  G.xl = g->ny * nc;
  G.n = (size_t)g->nx * g->ny;
  G.two_d = g->ny > 1;
  const int nx = g->nx, ny = g->ny, M = g->order_M, bc = g->bc;
  const size_t n = G.n;
  // variable-step BDF2 (w = omega): v^{n+1} - beta dt F = rc0 v^n + rc1 v^{n-1},
  // beta = (1+w)/(1+2w), rc0 = (1+w)^2/(1+2w), rc1 = -w^2/(1+2w)
  const bool var = bdf2 && !bdf3 && omega != 1.0;
  const double beta = !bdf2 ? 1.0 : (bdf3 ? 6.0 / 11.0 : (var ? (1.0 + omega) / (1.0 + 2.0 * omega) : 2.0 / 3.0));
  const StepParams sp = step_params(p->eps, p->dt, beta, p->sigma0);
  const double al1 = 1.0 / sqrt(sp.s1), al2 = 1.0 / sqrt(sp.s2);
  const double hx = spacing(bc, nx, g->x0, g->x1);
  const double hy = G.two_d ? spacing(bc, ny, g->y0, g->y1) : 1.0;
  G.cx1 = make_line(nx, bc, M, al1, hx);
  G.cx2 = make_line(nx, bc, M, al2, hx);
  if (G.two_d) {
    G.cy1 = make_line(ny, bc, M, al1, hy);
    G.cy2 = make_line(ny, bc, M, al2, hy);
  }

  // Dirichlet walls: the line inverses no longer preserve constants, so the
  // step runs in the shifted variable of eq. CahnHilliard_v (v = u + 1; the
  // vector model's v = u - z3), whose walls are homogeneous.  The caller's
  // field and histories are shifted in place for the step and back after it.
  const bool vform = bc == MOLT_BC_DIRICHLET;
  double ush[2] = {0.0, 0.0};
  if (vform) {
    ush[0] = vch ? -0.5 : -1.0;
    ush[1] = vch ? -0.5 * sqrt(3.0) : 0.0;
    HIPCHK(launch_addc(prec, d_u, -ush[0], -ush[1], n, nc, s));
    if (d_u_prev) HIPCHK(launch_addc(prec, d_u_prev, -ush[0], -ush[1], n, nc, s));
    if (d_u_prev2) HIPCHK(launch_addc(prec, d_u_prev2, -ush[0], -ush[1], n, nc, s));
  }

  HIPCHK(launch_state_init(st, p->tol, p->max_iter, p->fixed_iters, s));
  // rhs of the stepper
  PassArgs ra;
  memset(&ra, 0, sizeof(ra));
  ra.bdf2 = bdf2 ? (bdf3 ? 3 : (var ? 2 : 1)) : 0;
  ra.rc0 = (1.0 + omega) * (1.0 + omega) / (1.0 + 2.0 * omega);
  ra.rc1 = -omega * omega / (1.0 + 2.0 * omega);
  const size_t nel = n * nc;
  const void* base = nullptr;     // the iterate of the full form (precision prec)
  const void* base64 = nullptr;   // its FP64 value (hybrid)
  int it = 0;
  if (!L.hybrid) {
    ra.in[0] = d_u;
    ra.in[1] = bdf2 ? d_u_prev : d_u;
    ra.in[2] = bdf3 ? d_u_prev2 : d_u;
    MOLT_RC(enqueue_rhs(prec, G, ra, F, tot, jln, st, s));
    base = p->init == MOLT_INIT_LINEAR ? F[F_R] : d_u;
  } else {
    // FP64 shadow: R (the FP64 kernels read the FP32 fields, widening each
    // value exactly) and the first iteration in FP64, then the iterate
    // re-based and the increment narrowed for the FP32 iterations
    ra.in[0] = d_u;
    ra.in[1] = bdf2 ? d_u_prev : d_u;
    ra.in[2] = bdf3 ? d_u_prev2 : d_u;
    MOLT_RC(enqueue_rhs(MOLT_F64, G, ra, F64, w + L.tot64, w + L.jln64, st, s, PROG_RHSW));
    base64 = F64[F_R];
    if (p->init != MOLT_INIT_LINEAR) {  // the first iterate is u^n itself, in FP64
      void* u64 = w + L.in64[0];
      HIPCHK(launch_widen(u64, d_u, nel, s));
      base64 = u64;
    }
    // the FP32 iterations' base is the first iterate rounded to FP32, their
    // running sum starts at its rounding error (written by the iteration's P4)
    MOLT_RC(enqueue_iteration(MOLT_F64, G, sp, ush, 0, base64, F64, w + L.tot64, w + L.jln64, st, rpart, false, s,
                              F));
    base = F[F_R];
    it = 1;
  }
  // history: u^{n-1} -> u_prev2, u^n -> u_prev (after the rhs has consumed them)
  if (d_u_prev2 && d_u_prev) HIPCHK(launch_copy(prec, d_u_prev2, d_u_prev, nel, s));
  if (d_u_prev) HIPCHK(launch_copy(prec, d_u_prev, d_u, nel, s));
  // (init PREV: the iterate's base is u^n, which the history copy above has
  // just saved; d_u itself is overwritten only by the final result)

  const int fixed = p->fixed_iters;
  const int cap = fixed > 0 ? fixed : p->max_iter;
  // iterations are enqueued in batches between host checks of the device
  // state (2..32 iterations): up to a hint -- the previous step's count, from
  // the caller or the last step run in this workspace -- the batches end at
  // the hint, since counts change slowly from step to step; past it a batch
  // grows with the iterations already done (a quarter of them), so a step
  // that converges in a few iterations queues few that exit at once, and a
  // long one checks rarely
  if (iter_hint <= 0) iter_hint = workspace_hint(d_work);
  auto next_batch = [&](int done_its) {
    const int b = iter_hint > done_its ? iter_hint - done_its : done_its / 4;
    return b < 2 ? 2 : (b > 32 ? 32 : b);
  };
  int batch = next_batch(it);
  DevState* pin = state_readback();
  if (pin == nullptr) return fail(MOLT_EHIP, "hipHostMalloc of the state read-back failed");
  DevState& hst = *pin;
  memset(&hst, 0, sizeof(hst));
  for (;;) {
    const int nb = batch < cap - it ? batch : cap - it;
    for (int b = 0; b < nb; ++b, ++it) {
      if (L.hybrid && it % kRestartEvery == 0) {
        // FP64 restart: the full form from the iterate, then re-based
        void* v64 = F64[F_HIST];
        HIPCHK(launch_iterate64(v64, F[F_R], F[F_W], st, nel, s));
        MOLT_RC(enqueue_iteration(MOLT_F64, G, sp, ush, 0, v64, F64, w + L.tot64, w + L.jln64, st, rpart, false, s,
                                  F));
        continue;
      }
      // a whole run of increment iterations with no restart in it: one graph launch
      const int next_restart = L.hybrid ? (it / kRestartEvery + 1) * kRestartEvery : INT32_MAX;
      if (it > 0 && nb - b >= kIterRun && it + kIterRun <= next_restart) {
        hipGraphExec_t ex = iteration_graph(prec, G, sp, ush, base, F, tot, jln, st, rpart);
        if (ex != nullptr) {
          HIPCHK(hipGraphLaunch(ex, s));
          b += kIterRun - 1;
          it += kIterRun - 1;
          continue;
        }
      }
      MOLT_RC(enqueue_iteration(prec, G, sp, ush, it == 0 ? 0 : 1, base, F, tot, jln, st, rpart, true, s));
    }
    // the batch's last iteration is closed before its state is read
    HIPCHK(launch_close_pending(rpart, st, s));
    HIPCHK(hipMemcpyAsync(&hst, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (g_prof_on) prof_drain();
    if (hst.done || it >= cap) break;
    batch = next_batch(it);
  }
  HIPCHK(launch_finalize(prec, d_u, base, F[F_W], nel, s));
  if (vform) {
    HIPCHK(launch_addc(prec, d_u, ush[0], ush[1], n, nc, s));
    if (d_u_prev) HIPCHK(launch_addc(prec, d_u_prev, ush[0], ush[1], n, nc, s));
    if (d_u_prev2) HIPCHK(launch_addc(prec, d_u_prev2, ush[0], ush[1], n, nc, s));
  }
  if (vch)
    HIPCHK(launch_diag_vch(prec, d_u, nx, ny, bc, hx, hy, p->eps, partials, st, s));
  else
    HIPCHK(launch_diag(prec, d_u, nx, ny, bc, hx, hy, p->eps, partials, st, s));
  HIPCHK(hipMemcpyAsync(&hst, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (g_prof_on) prof_drain();
  workspace_hint_set(d_work, hst.iters);
  const bool conv = fixed > 0 || hst.last_resid < p->tol;
  if (info) {
    info->iters = hst.iters;
    info->converged = conv ? 1 : 0;
    info->residual = hst.last_resid;
    info->mass = hst.mass;
    info->energy = hst.energy;
    info->s1 = sp.s1;
    info->s2 = sp.s2;
    info->sigma = sp.sigma;
    info->mass2 = hst.mass2;
  }
  return conv ? MOLT_OK : MOLT_NOT_CONVERGED;
}

// SDIRK2 (Sec. 4.2, eta = 1 - sqrt(2)/2), the start-up of BDF3: written for the
// stage values V1 = v^n + eta dt K1, V2 = W + eta dt K2 with
// W = v^n + (1-eta) dt K1, the two stage equations are BE steps of size
// eta dt, from v^n and from W = v^n + ((1-eta)/eta)(V1 - v^n); v^{n+1} = V2.
// The histories (if given) are rotated: u_prev2 <- u_prev, u_prev <- u^n.
static int32_t sdirk2_impl(const molt_grid* g, const molt_ch_params* p, void* d_u, void* d_u_prev,
                           void* d_u_prev2, void* d_work, size_t work_bytes, molt_step_info* info, hipStream_t s) {
  const int prec = p->precision;
  const int nc = ncomp_of(p);
  const Layout L = ch_layout(g, prec, nc, true);
  if (!d_work || work_bytes < L.total) return fail(MOLT_EWORKSPACE, "workspace smaller than ch_workspace_bytes()");
  const size_t nel = (size_t)g->nx * g->ny * nc;
  void* stage = (char*)d_work + L.fld[F_STAGE];
  const double eta = 1.0 - sqrt(2.0) / 2.0;
  molt_ch_params q = *p;
  q.dt = eta * p->dt;
  molt_step_info i1, i2;
  HIPCHK(launch_copy(prec, stage, d_u, nel, s));
  int32_t rc1 = step_impl(g, &q, stage, nullptr, false, d_work, work_bytes, &i1, s, 0);
  if (rc1 < 0) return rc1;
  if (d_u_prev2 && d_u_prev) HIPCHK(launch_copy(prec, d_u_prev2, d_u_prev, nel, s));
  if (d_u_prev) HIPCHK(launch_copy(prec, d_u_prev, d_u, nel, s));
  HIPCHK(launch_lerp(prec, d_u, d_u, stage, (1.0 - eta) / eta, nel, s));
  int32_t rc2 = step_impl(g, &q, d_u, nullptr, false, d_work, work_bytes, &i2, s, 0);
  if (rc2 < 0) return rc2;
  if (info) {
    *info = i2;
    info->iters = i1.iters + i2.iters;
    info->converged = i1.converged && i2.converged;
  }
  return (rc1 == MOLT_NOT_CONVERGED || rc2 == MOLT_NOT_CONVERGED) ? MOLT_NOT_CONVERGED : MOLT_OK;
}

static int32_t check_params(const molt_ch_params* p) {
  if (!p) return fail(MOLT_EINVAL, "params is NULL");
  if (!(p->eps > 0) || !(p->dt > 0)) return fail(MOLT_EINVAL, "eps and dt must be positive");
  if (!(p->sigma0 > 0)) return fail(MOLT_EINVAL, "sigma0 must be positive");
  if (p->stepper != MOLT_BE && p->stepper != MOLT_BDF2 && p->stepper != MOLT_BDF3)
    return fail(MOLT_EINVAL, "unknown stepper");
  if (p->init != MOLT_INIT_PREV && p->init != MOLT_INIT_LINEAR) return fail(MOLT_EINVAL, "unknown init");
  if (p->fixed_iters < 0) return fail(MOLT_EINVAL, "fixed_iters must be >= 0");
  if (p->model != MOLT_MODEL_CH && p->model != MOLT_MODEL_VCH) return fail(MOLT_EINVAL, "unknown model");
  if (p->fixed_iters == 0 && (p->max_iter < 1 || !(p->tol >= 0))) return fail(MOLT_EINVAL, "need max_iter >= 1 and tol >= 0");
  if (p->model == MOLT_MODEL_VCH && p->stepper == MOLT_BDF3)
    return fail(MOLT_EUNSUPPORTED, "the vector model takes BE or BDF2");
  return MOLT_OK;
}

// the adaptive driver runs its own BE-BDF2 pair: the stepper asked for is not checked
static int32_t check_adapt_params(const molt_ch_params* p) {
  if (!p) return fail(MOLT_EINVAL, "params is NULL");
  molt_ch_params q = *p;
  q.stepper = MOLT_BDF2;
  return check_params(&q);
}

// --------------------------------------------------------------------------
// batched instances
// --------------------------------------------------------------------------
#define MOLT_BATCH_PREC(call) (prec == MOLT_F64 ? call##_f64 : call##_f32)
static hipError_t launch_batch_y(int prec, int K, int M, bool per, int pass, const SlotDesc* sd,
                                 const SlotCtl* ctl, const BlkMap* map, int nblk, hipStream_t s) {
  return MOLT_BATCH_PREC(launch_batch_y)(K, M, per, pass, sd, ctl, map, nblk, s);
}
static hipError_t launch_batch_comb(int prec, int pass, const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* map,
                                    int nblk, hipStream_t s) {
  return MOLT_BATCH_PREC(launch_batch_comb)(pass, sd, ctl, map, nblk, s);
}
static hipError_t launch_batch_x(int prec, int K, int M, bool per, int pass, const SlotDesc* sd, const SlotCtl* ctl,
                                 const BlkMap* map, int nblk, hipStream_t s) {
  return MOLT_BATCH_PREC(launch_batch_x)(K, M, per, pass, sd, ctl, map, nblk, s);
}
static hipError_t launch_batch_tail(int prec, const SlotDesc* sd, SlotCtl* ctl, const BlkMap* slots, int nslots,
                                    const BlkMap* pmap, int npblk, bool close_only, bool hybrid, hipStream_t s) {
  return MOLT_BATCH_PREC(launch_batch_tail)(sd, ctl, slots, nslots, pmap, npblk, close_only, hybrid, s);
}
static hipError_t launch_batch_react(int prec, const SlotDesc* sd, const SlotCtl* ctl, const BlkMap* pmap, int npblk,
                                     hipStream_t s) {
  return MOLT_BATCH_PREC(launch_batch_react)(sd, ctl, pmap, npblk, s);
}
static hipError_t launch_batch_init(int prec, const SlotDesc* sd, SlotCtl* ctl, int nslots, hipStream_t s) {
  return MOLT_BATCH_PREC(launch_batch_init)(sd, ctl, nslots, s);
}
static hipError_t launch_batch_count(int prec, const SlotCtl* ctl, int nslots, int* out, hipStream_t s) {
  return MOLT_BATCH_PREC(launch_batch_count)(ctl, nslots, out, s);
}
#undef MOLT_BATCH_PREC
struct BatchGroup {
  int K, M, per;
  size_t off;  // first map entry
  int nblk;
};

struct BatchPlan {
  int prec = 0;
  std::vector<size_t> slot_off;  // workspace offset of each slot's problem workspace
  std::vector<Layout> lay;
  std::vector<size_t> rec_first;  // first record of each slot
  size_t nrec = 0;
  size_t desc = 0, ctl = 0, rec = 0, map = 0, cnt = 0, total = 0;
  size_t nmap = 0;          // capacity of the map area in entries
  long long max_ticks = 0;  // upper bound of the ticks any slot needs (plain rounds)
  long long max_steps = 0;  // most steps of any slot (lean rounds add up to 2 rounds a step)
};

// Block maps of the slots in `act` (ascending): per-group ranges of one map.
// An FP32 batch is hybrid: its R phases and first iterations run the FP64
// kernels, grouped by the FP64 shapes (yg64, xg64).
struct BatchMaps {
  bool any_vch = false;  // a vector-model slot is listed: the tick runs the reaction pass
  bool any_prev = false; // an init-PREV slot is listed: a hybrid tick widens u^n for it
  bool hybrid = false;
  std::vector<BatchGroup> yg, xg, yg64, xg64;
  size_t comb_off = 0, pt_off = 0, sl_off = 0;
  int comb_n = 0, pt_n = 0, sl_n = 0;
  std::vector<BlkMap> map;
};

static int32_t check_instance(const molt_instance& in, int prec) {
  int32_t rc = check_params(&in.params);
  if (rc != MOLT_OK) return rc;
  if (in.params.precision != prec) return fail(MOLT_EINVAL, "all instances of a batch must use one precision");
  rc = check_grid(&in.grid, prec);
  if (rc != MOLT_OK) return rc;
  if (in.grid.ny < 2) return fail(MOLT_EUNSUPPORTED, "batched instances must be two-dimensional");
  if (in.grid.bc == MOLT_BC_DIRICHLET) return fail(MOLT_EUNSUPPORTED, "batched instances take periodic or Neumann boundaries");
  if (in.params.stepper == MOLT_BDF3) return fail(MOLT_EUNSUPPORTED, "batched instances take BE or BDF2");
  if (!in.d_u) return fail(MOLT_EINVAL, "instance field is NULL");
  if (in.nsteps < 0 || in.nsteps > 0x7fffffffLL) return fail(MOLT_EINVAL, "nsteps out of range");
  return MOLT_OK;
}

// y-passes are grouped by (M, boundary kind), x-passes by (K, M, boundary
// kind); the combine, pointwise and per-slot kernels take every listed slot.
// y-pass and x-pass groups of one precision's shapes, appended to the map
static void batch_pass_groups(const molt_instance* inst, const std::vector<int>& act, int prec,
                              std::vector<BlkMap>& m, std::vector<BatchGroup>& yg, std::vector<BatchGroup>& xg) {
  const int ks[4] = {4, 8, 16, 32};
  yg.clear();
  xg.clear();
  for (int kk = 0; kk < 3; ++kk)
    for (int M = 2; M <= 6; M += 2)
      for (int per = 1; per >= 0; --per) {
        BatchGroup g{ks[kk], M, per, m.size(), 0};
        for (int i : act) {
          const molt_grid& gr = inst[i].grid;
          if (gr.order_M != M || (gr.bc == MOLT_BC_PERIODIC) != (per == 1)) continue;
          if (ypass_pick_k(gr.ny, prec) != ks[kk]) continue;
          int nth, nseg;
          ypass_shape(prec, gr.ny, &nth, &nseg);
          const int nb = ((gr.nx + 63) / 64) * nseg * ncomp_of(&inst[i].params);
          for (int b = 0; b < nb; ++b) m.push_back(BlkMap{i, b});
        }
        g.nblk = (int)(m.size() - g.off);
        if (g.nblk > 0) yg.push_back(g);
      }
  for (int kk = 0; kk < 4; ++kk)
    for (int M = 2; M <= 6; M += 2)
      for (int per = 1; per >= 0; --per) {
        BatchGroup g{ks[kk], M, per, m.size(), 0};
        for (int i : act) {
          const molt_grid& gr = inst[i].grid;
          if (gr.order_M != M || (gr.bc == MOLT_BC_PERIODIC) != (per == 1)) continue;
          const int K = xpass_pick_k256(gr.nx, prec);
          if (K != ks[kk]) continue;
          const int lpb = 256 / xpass_tl(gr.nx, K);
          const int lines = gr.ny * ncomp_of(&inst[i].params);
          const int nb = (lines + lpb - 1) / lpb;
          for (int b = 0; b < nb; ++b) m.push_back(BlkMap{i, b});
        }
        g.nblk = (int)(m.size() - g.off);
        if (g.nblk > 0) xg.push_back(g);
      }
}

// y-passes are grouped by (K, M, boundary kind), x-passes by (K, M, boundary
// kind); the combine, pointwise and per-slot kernels take every listed slot.
static void batch_maps(const molt_instance* inst, const std::vector<int>& act, int prec, BatchMaps& B) {
  B.map.clear();
  B.any_vch = false;
  B.any_prev = false;
  B.hybrid = prec == MOLT_F32;
  for (int i : act) B.any_vch = B.any_vch || inst[i].params.model == MOLT_MODEL_VCH;
  for (int i : act) B.any_prev = B.any_prev || inst[i].params.init != MOLT_INIT_LINEAR;
  std::vector<BlkMap>& m = B.map;
  batch_pass_groups(inst, act, prec, m, B.yg, B.xg);
  B.yg64.clear();
  B.xg64.clear();
  if (B.hybrid) batch_pass_groups(inst, act, MOLT_F64, m, B.yg64, B.xg64);
  B.comb_off = m.size();
  for (int i : act) {
    const int nb = 2 * ((inst[i].grid.nx + 63) / 64) * ncomp_of(&inst[i].params);
    for (int b = 0; b < nb; ++b) m.push_back(BlkMap{i, b});
  }
  B.comb_n = (int)(m.size() - B.comb_off);
  B.pt_off = m.size();
  for (int i : act) {
    const int nb = diag_blocks((size_t)inst[i].grid.nx * inst[i].grid.ny);
    for (int b = 0; b < nb; ++b) m.push_back(BlkMap{i, b});
  }
  B.pt_n = (int)(m.size() - B.pt_off);
  B.sl_off = m.size();
  for (int i : act) m.push_back(BlkMap{i, 0});
  B.sl_n = (int)(m.size() - B.sl_off);
}

// map entries one instance can need under any shape of the table (both
// precisions' pass maps for an FP32 instance)
static size_t map_entries_max(const molt_instance& in, int prec) {
  const molt_grid& gr = in.grid;
  const int nc = ncomp_of(&in.params);
  const int ycols = (gr.nx + 63) / 64;
  size_t e = 2 * (size_t)ycols * nc + (size_t)diag_blocks((size_t)gr.nx * gr.ny) + 1;
  for (int pr = prec; ; pr = MOLT_F64) {
    const int lpb = 256 / xpass_tl(gr.nx, xpass_min_k(gr.nx, pr));
    e += ((size_t)ycols * ypass_max_segments(gr.ny) + (size_t)((gr.ny + lpb - 1) / lpb)) * nc;
    if (pr == MOLT_F64) break;
  }
  return e;
}

// Workspace layout of a batch; the map area holds the maps of every slot (the
// maps of any subset are shorter).
static int32_t batch_plan(const molt_instance* inst, int count, BatchPlan& P) {
  if (!inst || count < 1 || count > 65535) return fail(MOLT_EINVAL, "count must be in 1..65535");
  P.prec = inst[0].params.precision;
  const int prec = P.prec;
  size_t off = 0;
  P.slot_off.resize(count);
  P.lay.resize(count);
  P.rec_first.resize(count);
  P.nrec = 0;
  P.max_ticks = 0;
  P.max_steps = 0;
  size_t nmap = 0;
  for (int i = 0; i < count; ++i) {
    const int32_t rc = check_instance(inst[i], prec);
    if (rc != MOLT_OK) return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
    const int nc = ncomp_of(&inst[i].params);
    P.lay[i] = ch_layout(&inst[i].grid, prec, nc);
    P.slot_off[i] = off;
    off += al256(P.lay[i].total);
    P.rec_first[i] = P.nrec;
    P.nrec += (size_t)inst[i].nsteps;
    const molt_ch_params& p = inst[i].params;
    const long long cap = p.fixed_iters > 0 ? p.fixed_iters : p.max_iter;
    const long long ticks = (long long)inst[i].nsteps * (cap + 1);
    if (ticks > P.max_ticks) P.max_ticks = ticks;
    if (inst[i].nsteps > P.max_steps) P.max_steps = inst[i].nsteps;
    // map entries of the most fine-grained shapes the table allows
    nmap += map_entries_max(inst[i], prec);
  }
  if (nmap > 0x7fffffffULL) return fail(MOLT_EUNSUPPORTED, "batch too large");
  P.desc = off;
  off += al256((size_t)count * sizeof(SlotDesc));
  P.ctl = off;
  off += al256((size_t)count * sizeof(SlotCtl));
  P.rec = off;
  off += al256(P.nrec * sizeof(molt_step_info));
  P.cnt = off;
  off += 256;
  P.map = off;
  P.nmap = nmap;
  off += al256(nmap * sizeof(BlkMap));
  P.total = off;
  return MOLT_OK;
}

static void fill_slot(const molt_instance& in, const Layout& L, char* w, molt_step_info* rec, SlotDesc& d) {
  memset(&d, 0, sizeof(d));
  const molt_grid& g = in.grid;
  const molt_ch_params& p = in.params;
  const int prec = p.precision;
  const size_t esz = prec == MOLT_F64 ? 8 : 4;
  const double hx = spacing(g.bc, g.nx, g.x0, g.x1), hy = spacing(g.bc, g.ny, g.y0, g.y1);
  for (int v = 0; v < 2; ++v) {
    // v = 1 (BDF2) only differs for a BDF2 instance after its start-up step
    const double beta = (v == 1 && p.stepper == MOLT_BDF2) ? 2.0 / 3.0 : 1.0;
    const StepParams sp = step_params(p.eps, p.dt, beta, p.sigma0);
    const double al[2] = {1.0 / sqrt(sp.s1), 1.0 / sqrt(sp.s2)};
    for (int k = 0; k < 2; ++k) {
      d.cx[v][k] = make_line(g.nx, g.bc, g.order_M, al[k], hx);
      d.cy[v][k] = make_line(g.ny, g.bc, g.order_M, al[k], hy);
    }
    d.sigma[v] = sp.sigma;
    d.kappa[v] = sp.a / sp.s1;
    d.s1[v] = sp.s1;
    d.s2[v] = sp.s2;
  }
  d.u = in.d_u;
  for (int f = 0; f < F_COUNT; ++f) d.fld[f] = w + L.fld[f];
  d.tot = w + L.tot;
  d.jln = w + L.jln;
  d.st = (DevState*)(w + L.state);
  d.rpart = (double*)(w + L.rpart);
  d.partials = (double*)(w + L.partials);
  d.rec = rec;
  d.hx = hx;
  d.hy = hy;
  d.eps = p.eps;
  d.area = hx * hy;
  d.tol = p.tol;
  d.nx = g.nx;
  d.ny = g.ny;
  d.bc = g.bc;
  d.M = g.order_M;
  d.stepper = p.stepper;
  d.init = p.init;
  d.nsteps = (int32_t)in.nsteps;
  d.max_iter = p.max_iter;
  d.fixed = p.fixed_iters;
  const int K = xpass_pick_k256(g.nx, prec);
  d.tlx = xpass_tl(g.nx, K);
  d.vecx = ((size_t)g.nx * esz) % 16 == 0 && (uintptr_t)in.d_u % 16 == 0 && (uintptr_t)w % 16 == 0;
  d.model = p.model;
  d.ncomp = ncomp_of(&p);
  d.xblocks = (g.ny * d.ncomp + 256 / d.tlx - 1) / (256 / d.tlx);
  ypass_shape(prec, g.ny, &d.ynth, &d.ynseg);
  d.yk = ypass_pick_k(g.ny, prec);
  d.ycols = (g.nx + 63) / 64;
  d.dblocks = diag_blocks((size_t)g.nx * g.ny);
  d.hybrid = L.hybrid ? 1 : 0;
  if (L.hybrid) {
    for (int f = 0; f < F_COUNT; ++f) d.fld64[f] = w + L.fld64[f];
    d.tot64 = w + L.tot64;
    d.jln64 = w + L.jln64;
    d.u64 = w + L.in64[0];
    d.hist64 = w + L.in64[1];
    const int K64 = xpass_pick_k256(g.nx, MOLT_F64);
    d.tlx64 = xpass_tl(g.nx, K64);
    d.vecx64 = ((size_t)g.nx * 8) % 16 == 0 && (uintptr_t)w % 16 == 0;
    d.xblocks64 = (g.ny * d.ncomp + 256 / d.tlx64 - 1) / (256 / d.tlx64);
    ypass_shape(MOLT_F64, g.ny, &d.ynth64, &d.ynseg64);
    d.yk64 = ypass_pick_k(g.ny, MOLT_F64);
  }
}

// close_only: the iteration's close without the step finish and phase update
// (lean ticks: a round of lean ticks ends with one full tick)
static hipError_t batch_tick(int prec, const BatchMaps& B, const SlotDesc* sd, SlotCtl* ctl, const BlkMap* map,
                             hipStream_t s, bool close_only = false) {
  hipError_t e;
  // a hybrid batch runs every pass in the FP64 kernels (slots in their R phase
  // or first iteration) and in the FP32 kernels (the others)
  const int nprec = B.hybrid ? 2 : 1;
  const int precs[2] = {B.hybrid ? MOLT_F64 : prec, prec};
  if (B.hybrid && B.any_prev && (e = launch_batch_widen(sd, ctl, map + B.pt_off, B.pt_n, s)) != hipSuccess) return e;
  for (int k = 0; k < nprec && B.any_vch; ++k)
    if ((e = launch_batch_react(precs[k], sd, ctl, map + B.pt_off, B.pt_n, s)) != hipSuccess) return e;
  for (int pass = 1; pass <= 3; pass += 2) {
    for (int k = 0; k < nprec; ++k) {
      const int pr = precs[k];
      const std::vector<BatchGroup>& yg = (B.hybrid && k == 0) ? B.yg64 : B.yg;
      for (const BatchGroup& g : yg)
        if ((e = launch_batch_y(pr, g.K, g.M, g.per != 0, pass, sd, ctl, map + g.off, g.nblk, s)) != hipSuccess)
          return e;
      if ((e = launch_batch_comb(pr, pass, sd, ctl, map + B.comb_off, B.comb_n, s)) != hipSuccess) return e;
    }
    for (int k = 0; k < nprec; ++k) {
      const int pr = precs[k];
      const std::vector<BatchGroup>& xg = (B.hybrid && k == 0) ? B.xg64 : B.xg;
      for (const BatchGroup& g : xg)
        if ((e = launch_batch_x(pr, g.K, g.M, g.per != 0, pass + 1, sd, ctl, map + g.off, g.nblk, s)) != hipSuccess)
          return e;
    }
  }
  return launch_batch_tail(prec, sd, ctl, map + B.sl_off, B.sl_n, map + B.pt_off, B.pt_n, close_only, B.hybrid, s);
}

// `ticks` ticks and the active-slot count, captured as one executable graph
static hipError_t capture_round(int prec, const BatchMaps& B, const SlotDesc* sd, SlotCtl* ctl, const BlkMap* map,
                                int count, int* dcnt, int ticks, bool lean, hipStream_t s, hipGraphExec_t* exec) {
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  for (int k = 0; k < ticks && e == hipSuccess; ++k) e = batch_tick(prec, B, sd, ctl, map, s, lean && k < ticks - 1);
  if (e == hipSuccess) e = launch_batch_count(prec, ctl, count, dcnt, s);
  const hipError_t e2 = hipStreamEndCapture(s, &graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  return e;
}

static int32_t solve_batch_impl(const molt_instance* inst, int count, void* d_work, size_t work_bytes,
                                molt_step_info* per_step, hipStream_t s) {
  BatchPlan P;
  int32_t rc = batch_plan(inst, count, P);
  if (rc != MOLT_OK) return rc;
  if (!d_work || work_bytes < P.total) return fail(MOLT_EWORKSPACE, "workspace smaller than ch_batch_workspace_bytes()");
  const int prec = P.prec;
  char* w = (char*)d_work;
  std::vector<SlotDesc> descs(count);
  molt_step_info* drec = (molt_step_info*)(w + P.rec);
  for (int i = 0; i < count; ++i) fill_slot(inst[i], P.lay[i], w + P.slot_off[i], drec + P.rec_first[i], descs[i]);
  SlotDesc* sd = (SlotDesc*)(w + P.desc);
  SlotCtl* ctl = (SlotCtl*)(w + P.ctl);
  BlkMap* map = (BlkMap*)(w + P.map);
  int* dcnt = (int*)(w + P.cnt);
  std::vector<int> act;
  for (int i = 0; i < count; ++i)
    if (inst[i].nsteps > 0) act.push_back(i);
  BatchMaps B;
  batch_maps(inst, act, prec, B);
  if (B.map.size() > P.nmap) return fail(MOLT_EHIP, "internal: batch maps exceed their area");
  HIPCHK(hipMemcpyAsync(sd, descs.data(), (size_t)count * sizeof(SlotDesc), hipMemcpyHostToDevice, s));
  if (!B.map.empty())
    HIPCHK(hipMemcpyAsync(map, B.map.data(), B.map.size() * sizeof(BlkMap), hipMemcpyHostToDevice, s));
  HIPCHK(launch_batch_init(prec, sd, ctl, count, s));

  const int ticks = g_batch_ticks;
  const bool use_graph = g_batch_graph && s != nullptr && !g_prof_on;
  // two pinned words and events: round r's active count is read while round
  // r+1 runs
  static thread_local int* pin = nullptr;
  if (!pin && hipHostMalloc((void**)&pin, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    pin = nullptr;
    return fail(MOLT_EHIP, "hipHostMalloc of the batch status words failed");
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t exec = nullptr;
  std::string err;
  for (int b = 0; b < 2 && err.empty(); ++b)
    if (hipEventCreateWithFlags(&ev[b], hipEventDisableTiming) != hipSuccess) err = "hipEventCreate failed";
  std::vector<SlotCtl> hctl;
  // a lean round finishes a step only at its end: the R phase and the wait
  // after convergence take up to one round each
  const long long max_rounds = (P.max_ticks + 2LL * ticks * P.max_steps) / ticks + 3;
  long long rounds = 0, since = 0;  // rounds in all, rounds since the maps were last built
  int planned = (int)act.size();
  bool finished = act.empty();
  // with at most this many instances left, a round's ticks but the last run
  // only the iteration (no step finish): a converged instance waits for the
  // round's end to start its next step, but each iteration of a lone long
  // instance takes three kernel launches fewer
  const int lean_slots = g_batch_lean;
  bool lean = planned <= lean_slots;
  while (err.empty() && !finished) {
    hipError_t e = hipSuccess;
    if (use_graph && !exec) {
      e = capture_round(prec, B, sd, ctl, map, count, dcnt, ticks, lean, s, &exec);
      if (e != hipSuccess) {
        err = std::string("batched tick capture: ") + hipGetErrorString(e);
        break;
      }
    }
    const int b = (int)(since & 1);
    if (exec) {
      e = hipGraphLaunch(exec, s);
    } else {
      for (int k = 0; k < ticks && e == hipSuccess; ++k) e = batch_tick(prec, B, sd, ctl, map, s, lean && k < ticks - 1);
      if (e == hipSuccess) e = launch_batch_count(prec, ctl, count, dcnt, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&pin[b], dcnt, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(ev[b], s);
    if (e != hipSuccess) {
      err = std::string("batched round: ") + hipGetErrorString(e);
      break;
    }
    ++rounds;
    ++since;
    if (rounds > max_rounds) {
      err = "batched solve exceeded its tick bound";
      break;
    }
    if (since < 2) continue;
    e = hipEventSynchronize(ev[1 - b]);
    if (e != hipSuccess) {
      err = std::string("hipEventSynchronize: ") + hipGetErrorString(e);
      break;
    }
    if (g_prof_on) prof_drain();
    const int active = pin[1 - b];
    if (active == 0) {
      finished = true;
    } else if (2 * active <= planned) {
      // half the planned slots are idle: rebuild the maps for the others
      e = hipStreamSynchronize(s);
      hctl.resize(count);
      if (e == hipSuccess) e = hipMemcpy(hctl.data(), ctl, (size_t)count * sizeof(SlotCtl), hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        err = std::string("batch re-plan: ") + hipGetErrorString(e);
        break;
      }
      act.clear();
      for (int i = 0; i < count; ++i)
        if (hctl[i].phase != PH_IDLE) act.push_back(i);
      if (act.empty()) {
        finished = true;
        break;
      }
      batch_maps(inst, act, prec, B);
      e = hipMemcpy(map, B.map.data(), B.map.size() * sizeof(BlkMap), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        err = std::string("batch re-plan: ") + hipGetErrorString(e);
        break;
      }
      planned = (int)act.size();
      lean = planned <= lean_slots;
      since = 0;
      if (exec) {
        (void)hipGraphExecDestroy(exec);
        exec = nullptr;
      }
    }
  }
  const hipError_t es = hipStreamSynchronize(s);
  if (err.empty() && es != hipSuccess) err = std::string("hipStreamSynchronize: ") + hipGetErrorString(es);
  if (g_prof_on) prof_drain();
  for (int b = 0; b < 2; ++b)
    if (ev[b]) (void)hipEventDestroy(ev[b]);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (!err.empty()) return fail(MOLT_EHIP, err);
  int32_t status = MOLT_OK;
  std::vector<molt_step_info> rec(P.nrec);
  if (P.nrec > 0) {
    HIPCHK(hipMemcpyAsync(rec.data(), drec, P.nrec * sizeof(molt_step_info), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  for (size_t r = 0; r < P.nrec; ++r)
    if (!rec[r].converged) status = MOLT_NOT_CONVERGED;
  if (per_step && P.nrec > 0) memcpy(per_step, rec.data(), P.nrec * sizeof(molt_step_info));
  return status;
}

// --------------------------------------------------------------------------
// adaptive time steps (Sec. 6, Algorithm 1) with the BE-BDF2 estimator
// --------------------------------------------------------------------------
struct AdaptLayout {
  Layout step;     // the step driver's workspace (first)
  size_t fld[5];   // u_BE, candidate, u^{n-1}, trial history, u^n backup
  size_t part, out, total;
};

static AdaptLayout adapt_layout(const molt_grid* g, const molt_ch_params* p) {
  AdaptLayout A;
  const int nc = ncomp_of(p);
  A.step = ch_layout(g, p->precision, nc);
  const size_t fb = al256((size_t)g->nx * g->ny * nc * (p->precision == MOLT_F64 ? 8 : 4));
  size_t off = al256(A.step.total);
  for (int i = 0; i < 5; ++i) {
    A.fld[i] = off;
    off += fb;
  }
  A.part = off;
  off += al256((size_t)diag_blocks((size_t)g->nx * g->ny * nc) * sizeof(double));
  A.out = off;
  off += 256;
  A.total = off;
  return A;
}

// Algorithm 1's decision: accepted?, and the factor of the next trial step
static bool adapt_decide(double eta, double tol, int nit, int nmaxit, double theta, double gamma, double* fac) {
  const double grow = eta > 0.0 ? theta * sqrt(tol / eta) : INFINITY;
  if (eta <= tol) {
    const double r = (double)nit / (double)nmaxit;
    if (r < 0.7) {
      *fac = grow < gamma ? grow : gamma;
      return true;
    }
    if (r < 1.0) {
      *fac = grow < 1.0 ? grow : 1.0;
      return true;
    }
    *fac = 1.0 / gamma;
    return false;
  }
  *fac = eta / tol > 2.0 ? 1.0 / gamma : grow;
  return false;
}

static int32_t check_adapt(const molt_adapt_params* ap) {
  if (!ap) return fail(MOLT_EINVAL, "adaptive parameters are NULL");
  if (!(ap->t_end > 0) || !(ap->dt0 > 0) || !(ap->lte_tol > 0) || ap->nmaxit < 1 || !(ap->theta > 0) ||
      !(ap->gamma > 1) || !(ap->dt_min >= 0) || !(ap->dt_max > 0) || ap->max_attempts < 1)
    return fail(MOLT_EINVAL, "need t_end, dt0, lte_tol, theta, dt_max > 0, gamma > 1, nmaxit, max_attempts >= 1");
  return MOLT_OK;
}

static int32_t solve_adaptive_impl(const molt_grid* g, const molt_ch_params* p0, const molt_adapt_params* ap,
                                   void* d_u, void* d_work, size_t work_bytes, molt_adapt_record* rec,
                                   int32_t max_rec, int32_t* nrec, double* t_final, hipStream_t s) {
  const AdaptLayout A = adapt_layout(g, p0);
  if (!d_work || work_bytes < A.total)
    return fail(MOLT_EWORKSPACE, "workspace smaller than ch_adaptive_workspace_bytes()");
  const int prec = p0->precision;
  const size_t nel = (size_t)g->nx * g->ny * ncomp_of(p0);
  const size_t esz = prec == MOLT_F64 ? 8 : 4;
  char* w = (char*)d_work;
  void* ube = w + A.fld[0];
  void* cand = w + A.fld[1];
  void* uprev = w + A.fld[2];
  void* hist = w + A.fld[3];
  double* part = (double*)(w + A.part);
  double* dout = (double*)(w + A.out);
  molt_ch_params p = *p0;
  p.max_iter = ap->nmaxit;
  p.fixed_iters = 0;
  p.stepper = MOLT_BDF2;  // Algorithm 1 runs the BE-BDF2 pair whatever stepper was asked for
  double t = 0.0, dt = ap->dt0, dtprev = 0.0;
  bool have_prev = false;
  int32_t m = 0;
  int32_t status = MOLT_OK;
  const double tiny = 1e-14 * ap->t_end;
  for (int32_t k = 0; k < ap->max_attempts && t < ap->t_end - tiny; ++k) {
    dt = fmin(fmin(dt, ap->t_end - t), ap->dt_max);
    if (dt < ap->dt_min) {
      status = fail(MOLT_NOT_CONVERGED, "the time step fell below dt_min");
      break;
    }
    molt_step_info i1, i2, i3;
    memset(&i3, 0, sizeof(i3));
    int32_t rc;
    double eta;
    HIPCHK(hipMemcpyAsync(ube, d_u, nel * esz, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(cand, d_u, nel * esz, hipMemcpyDeviceToDevice, s));
    p.dt = dt;
    if (!have_prev) {
      // first step: Richardson (step-doubling) estimate of BE, keep the two half steps
      if ((rc = step_impl(g, &p, ube, nullptr, false, d_work, A.step.total, &i1, s, 0)) < 0) return rc;
      p.dt = 0.5 * dt;
      if ((rc = step_impl(g, &p, cand, nullptr, false, d_work, A.step.total, &i2, s, 0)) < 0) return rc;
      if ((rc = step_impl(g, &p, cand, nullptr, false, d_work, A.step.total, &i3, s, 0)) < 0) return rc;
      HIPCHK(launch_maxdiff(prec, ube, cand, nel, part, dout, s));
      HIPCHK(hipMemcpyAsync(&eta, dout, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      eta *= 0.5;
    } else {
      // BE and variable-step BDF2 from the same state; keep the BDF2 solution
      if ((rc = step_impl(g, &p, ube, nullptr, false, d_work, A.step.total, &i1, s, 0)) < 0) return rc;
      HIPCHK(hipMemcpyAsync(hist, uprev, nel * esz, hipMemcpyDeviceToDevice, s));
      if ((rc = step_impl(g, &p, cand, hist, true, d_work, A.step.total, &i2, s, 0, dt / dtprev)) < 0) return rc;
      HIPCHK(launch_maxdiff(prec, ube, cand, nel, part, dout, s));
      HIPCHK(hipMemcpyAsync(&eta, dout, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    int nit = i1.iters > i2.iters ? i1.iters : i2.iters;
    if (i3.iters > nit) nit = i3.iters;
    double fac = 1.0;
    const bool ok = adapt_decide(eta, ap->lte_tol, nit, ap->nmaxit, ap->theta, ap->gamma, &fac);
    if (rec && m < max_rec) {
      rec[m].t = t;
      rec[m].dt = dt;
      rec[m].eta = eta;
      rec[m].iters = nit;
      rec[m].accepted = ok ? 1 : 0;
      rec[m].energy = ok ? (have_prev ? i2.energy : i3.energy) : 0.0;
    }
    ++m;
    if (ok) {
      HIPCHK(hipMemcpyAsync(uprev, d_u, nel * esz, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(d_u, cand, nel * esz, hipMemcpyDeviceToDevice, s));
      t += dt;
      dtprev = dt;
      have_prev = true;
    }
    dt *= fac;
  }
  HIPCHK(hipStreamSynchronize(s));
  if (status == MOLT_OK && t < ap->t_end - tiny)
    status = fail(MOLT_NOT_CONVERGED, "max_attempts reached before t_end");
  if (nrec) *nrec = m;
  if (t_final) *t_final = t;
  return status;
}

// --------------------------------------------------------------------------
// serving: a resident batched engine that admits requests while others run
// --------------------------------------------------------------------------

static size_t footprint(const molt_instance& in, int prec) {
  return al256(ch_layout(&in.grid, prec, ncomp_of(&in.params)).total) +
         al256((size_t)in.nsteps * sizeof(molt_step_info));
}

static size_t server_map_cap(int max_slots, size_t pool_bytes) { return (size_t)max_slots * 64 + pool_bytes / 1024; }

}  // namespace molt

struct molt_server {
  struct Req {
    int64_t id;
    molt_instance inst;
  };
  struct Slot {
    bool used = false;
    int64_t id = 0;
    long long admit_round = 0;
    size_t off = 0, bytes = 0, map_need = 0;
  };
  int prec = 0, max_slots = 0;
  hipStream_t s = nullptr, cs = nullptr;  // work stream, record-copy stream
  char* w = nullptr;
  molt::SlotDesc* sd = nullptr;
  molt::SlotCtl* ctl = nullptr;
  molt::BlkMap* map = nullptr;
  size_t map_cap = 0, map_used = 0;
  size_t pool_off = 0, pool_end = 0;
  std::map<size_t, size_t> free_;  // pool: offset -> size of each free range
  std::vector<Slot> slots;
  std::vector<molt_instance> insts;  // by slot
  std::vector<int> free_slots;
  std::deque<Req> queue;
  std::deque<molt_result> done;
  molt::BatchMaps B;
  bool dirty = false;
  // pipeline of rounds: snapshots of the control words, one pinned buffer per round in flight
  molt::SlotCtl* pin[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  // pinned staging of uploads: one descriptor and control word per slot (a slot
  // is reused only after its rounds are retired), two map buffers with events
  molt::SlotDesc* up_desc = nullptr;
  molt::SlotCtl* up_ctl = nullptr;
  molt::BlkMap* up_map[2] = {nullptr, nullptr};
  hipEvent_t ev_map[2] = {nullptr, nullptr};
  int map_k = 0;
  long long round_of[2] = {-1, -1};
  long long rounds = 0;
  int inflight = 0, head = 0;
};

namespace molt {

static bool pool_alloc(molt_server* S, size_t bytes, size_t* off) {
  for (auto it = S->free_.begin(); it != S->free_.end(); ++it) {
    if (it->second < bytes) continue;
    *off = it->first;
    const size_t rest = it->second - bytes;
    const size_t roff = it->first + bytes;
    S->free_.erase(it);
    if (rest) S->free_[roff] = rest;
    return true;
  }
  return false;
}

static void pool_free(molt_server* S, size_t off, size_t bytes) {
  auto it = S->free_.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != S->free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    S->free_.erase(nx);
  }
  if (it != S->free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      S->free_.erase(it);
    }
  }
}

// retire the oldest round in flight: finished slots -> results, memory freed
static int32_t server_retire(molt_server* S) {
  const int b = S->head;
  HIPCHK(hipEventSynchronize(S->ev[b]));
  if (g_prof_on) prof_drain();
  const long long r = S->round_of[b];
  for (int i = 0; i < S->max_slots; ++i) {
    molt_server::Slot& sl = S->slots[i];
    if (!sl.used || sl.admit_round > r || S->pin[b][i].phase != PH_IDLE) continue;
    const molt_instance& in = S->insts[i];
    std::vector<molt_step_info> rec((size_t)in.nsteps);
    const Layout L = ch_layout(&in.grid, S->prec, ncomp_of(&in.params));
    molt_result res;
    memset(&res, 0, sizeof(res));
    res.id = sl.id;
    res.steps = (int32_t)in.nsteps;
    res.status = MOLT_OK;
    if (in.nsteps > 0) {
      HIPCHK(hipMemcpyAsync(rec.data(), S->w + sl.off + al256(L.total), rec.size() * sizeof(molt_step_info),
                            hipMemcpyDeviceToHost, S->cs));
      HIPCHK(hipStreamSynchronize(S->cs));
      for (const molt_step_info& x : rec) {
        res.iters += x.iters;
        if (!x.converged) res.status = MOLT_NOT_CONVERGED;
      }
      res.last = rec.back();
    }
    S->done.push_back(res);
    pool_free(S, sl.off, sl.bytes);
    S->map_used -= sl.map_need;
    sl = molt_server::Slot();
    S->free_slots.push_back(i);
    S->dirty = true;
  }
  S->head = 1 - b;
  --S->inflight;
  return MOLT_OK;
}

// admit queued requests (in order) while a slot, pool memory and map room are free
static int32_t server_admit(molt_server* S) {
  while (!S->queue.empty() && !S->free_slots.empty()) {
    const molt_server::Req& q = S->queue.front();
    const size_t need = footprint(q.inst, S->prec), mneed = map_entries_max(q.inst, S->prec);
    if (S->map_used + mneed > S->map_cap) break;
    size_t off = 0;
    if (!pool_alloc(S, need, &off)) break;
    const int i = S->free_slots.back();
    S->free_slots.pop_back();
    molt_server::Slot& sl = S->slots[i];
    sl.used = true;
    sl.id = q.id;
    sl.admit_round = S->rounds;
    sl.off = off;
    sl.bytes = need;
    sl.map_need = mneed;
    S->map_used += mneed;
    S->insts[i] = q.inst;
    const Layout L = ch_layout(&q.inst.grid, S->prec, ncomp_of(&q.inst.params));
    SlotDesc& d = S->up_desc[i];
    fill_slot(q.inst, L, S->w + off, (molt_step_info*)(S->w + off + al256(L.total)), d);
    SlotCtl& c = S->up_ctl[i];
    c.phase = q.inst.nsteps > 0 ? PH_R : PH_IDLE;
    c.step = 0;
    c.var = 0;
    c.fp64 = (S->prec == MOLT_F64 || c.phase == PH_R) ? 1 : 0;  // (as the device's slot_fp64_next)
    // stream order puts these after every round already queued
    HIPCHK(hipMemcpyAsync(S->sd + i, &d, sizeof(d), hipMemcpyHostToDevice, S->s));
    HIPCHK(hipMemcpyAsync(S->ctl + i, &c, sizeof(c), hipMemcpyHostToDevice, S->s));
    S->queue.pop_front();
    S->dirty = true;
  }
  return MOLT_OK;
}

static int server_active(const molt_server* S) {
  int a = 0;
  for (const molt_server::Slot& sl : S->slots) a += sl.used ? 1 : 0;
  return a;
}

static int32_t server_run(molt_server* S, int nrounds) {
  for (int r = 0; r < nrounds; ++r) {
    if (S->inflight == 2) {
      const int32_t rc = server_retire(S);
      if (rc != MOLT_OK) return rc;
    }
    int32_t rc = server_admit(S);
    if (rc != MOLT_OK) return rc;
    if (server_active(S) == 0) {
      while (S->inflight > 0)
        if ((rc = server_retire(S)) != MOLT_OK) return rc;
      rc = server_admit(S);
      if (rc != MOLT_OK) return rc;
      if (server_active(S) == 0) return MOLT_OK;
    }
    if (S->dirty) {
      std::vector<int> act;
      for (int i = 0; i < S->max_slots; ++i)
        if (S->slots[i].used) act.push_back(i);
      batch_maps(S->insts.data(), act, S->prec, S->B);
      if (S->B.map.size() > S->map_cap) return fail(MOLT_EHIP, "internal: server maps exceed their area");
      const int mb = S->map_k & 1;
      HIPCHK(hipEventSynchronize(S->ev_map[mb]));  // the upload that last used this buffer
      memcpy(S->up_map[mb], S->B.map.data(), S->B.map.size() * sizeof(BlkMap));
      HIPCHK(hipMemcpyAsync(S->map, S->up_map[mb], S->B.map.size() * sizeof(BlkMap), hipMemcpyHostToDevice, S->s));
      HIPCHK(hipEventRecord(S->ev_map[mb], S->s));
      ++S->map_k;
      S->dirty = false;
    }
    const int b = (S->head + S->inflight) & 1;
    hipError_t e = hipSuccess;
    for (int k = 0; k < g_batch_ticks && e == hipSuccess; ++k) e = batch_tick(S->prec, S->B, S->sd, S->ctl, S->map, S->s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S->pin[b], S->ctl, (size_t)S->max_slots * sizeof(SlotCtl), hipMemcpyDeviceToHost, S->s);
    if (e == hipSuccess) e = hipEventRecord(S->ev[b], S->s);
    if (e != hipSuccess) return fail(MOLT_EHIP, std::string("server round: ") + hipGetErrorString(e));
    S->round_of[b] = S->rounds++;
    ++S->inflight;
  }
  return MOLT_OK;
}

}  // namespace molt

using namespace molt;

// --------------------------------------------------------------------------
// the line inverse along one axis of `batch` stacked fields (shared by
// mol_t_helmholtz_sweep and its no-allocation variant)
// --------------------------------------------------------------------------
namespace molt {

int32_t set_error(int32_t code, const char* msg) { return fail(code, msg); }

int32_t sweep_check(const molt_grid* g, int32_t axis, double alpha, int32_t precision, const void* d_in,
                    const void* d_out, int64_t batch) {
  int32_t rc = check_grid(g, precision);
  if (rc != MOLT_OK) return rc;
  if (axis != 0 && axis != 1) return fail(MOLT_EINVAL, "axis must be 0 or 1");
  if (!(alpha > 0) || !isfinite(alpha)) return fail(MOLT_EINVAL, "alpha must be positive");
  if (batch < 1 || batch > 65535) return fail(MOLT_EINVAL, "batch must be in 1..65535");
  if (!d_in || !d_out) return fail(MOLT_EINVAL, "NULL field pointer");
  return MOLT_OK;
}

// y-pass scratch of a sweep under the current shape table: segment totals /
// seeds (one field, two directions, per segment and column) and the periodic
// closing-cell quadratures (one per column), each 256-byte aligned
void sweep_scratch_layout(const molt_grid* g, int32_t precision, int64_t batch, size_t* tot_bytes,
                          size_t* jln_bytes) {
  const size_t esz = precision == MOLT_F64 ? 8 : 4;
  int nth = 0, nseg = 0;
  ypass_shape(precision, g->ny, &nth, &nseg);
  *tot_bytes = al256((size_t)2 * nseg * g->nx * batch * esz);
  *jln_bytes = al256((size_t)g->nx * batch * esz);
}

// tot, jln: y-pass scratch (axis 1, ny > 1); cpy: a field-sized buffer for an
// in-place y sweep (NULL: in-place y sweeps are refused)
int32_t sweep_impl(const molt_grid* g, int32_t axis, double alpha, int32_t precision, const void* d_in, void* d_out,
                   int64_t batch, void* tot, void* jln, void* cpy, hipStream_t s) {
  const size_t n = (size_t)g->nx * g->ny;
  const size_t esz = precision == MOLT_F64 ? 8 : 4;
  PassArgs a;
  memset(&a, 0, sizeof(a));
  a.in[0] = d_in;
  a.out[0] = d_out;
  if (axis == 0) {
    const double hx = spacing(g->bc, g->nx, g->x0, g->x1);
    const LineCoef c = make_line(g->nx, g->bc, g->order_M, alpha, hx);
    const long long nlines = (long long)g->ny * batch;
    if (nlines > 0x7fffffffLL) return fail(MOLT_EUNSUPPORTED, "too many lines");
    HIPCHK(launch_xpass(precision, PROG_SWEEP, c, a, nullptr, (int)nlines, nullptr, s));
    return MOLT_OK;
  }
  if (g->ny == 1) {  // y-direction of a 1D problem: identity
    if (d_in != d_out) HIPCHK(hipMemcpyAsync(d_out, d_in, n * esz * batch, hipMemcpyDeviceToDevice, s));
    return MOLT_OK;
  }
  if (d_in == d_out) {  // neighbouring segments read each other's rows: sweep from a copy
    if (cpy == nullptr) return fail(MOLT_EINVAL, "an in-place y sweep needs a workspace copy of the field");
    HIPCHK(launch_copy(precision, cpy, d_in, n * batch, s));
    a.in[0] = cpy;
  }
  const double hy = spacing(g->bc, g->ny, g->y0, g->y1);
  const LineCoef c = make_line(g->ny, g->bc, g->order_M, alpha, hy);
  HIPCHK(launch_ypass(precision, PROG_SWEEP, c, a, nullptr, g->nx, (int)batch, tot, jln, false, s));
  return MOLT_OK;
}

}  // namespace molt

extern "C" {

const char* molt_strerror(int32_t status) {
  switch (status) {
    case MOLT_OK: return "ok";
    case MOLT_NOT_CONVERGED: return "fixed-point iteration reached max_iter";
    case MOLT_EINVAL: return "invalid argument";
    case MOLT_EUNSUPPORTED: return "unsupported configuration";
    case MOLT_EHIP: return "HIP runtime error";
    case MOLT_EWORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

const char* molt_last_error(void) { return g_err.c_str(); }

int32_t molt_set_option(int32_t option, int64_t value) {
  if (option == MOLT_OPT_BATCH_TICKS && value >= 1 && value <= 1024) {
    g_batch_ticks = (int)value;
    return MOLT_OK;
  }
  if (option == MOLT_OPT_BATCH_GRAPH && (value == 0 || value == 1)) {
    g_batch_graph = (int)value;
    return MOLT_OK;
  }
  if (option == MOLT_OPT_BATCH_LEAN && value >= 0 && value <= 1024) {
    g_batch_lean = (int)value;
    return MOLT_OK;
  }
  if (option == MOLT_OPT_STEP_GRAPH && (value == 0 || value == 1)) {
    g_iter_graph_on = value == 1;
    return MOLT_OK;
  }
  return fail(MOLT_EINVAL, "unknown option or value out of range");
}

int32_t molt_profile(int32_t enable) {
  prof_drain();
  for (int k = 0; k < kProfKinds; ++k) {
    g_prof_ms[k] = 0.0;
    g_prof_n[k] = 0;
  }
  g_prof_on = enable != 0;
  return MOLT_OK;
}

int32_t molt_profile_only(int32_t kind) {
  if (kind < -1 || kind >= kProfKinds) return fail(MOLT_EINVAL, "profile kind out of range");
  prof_drain();
  g_prof_only = kind;
  return MOLT_OK;
}

int32_t molt_profile_read(molt_prof_entry* out, int32_t max_entries) {
  if (!out || max_entries < 0) return fail(MOLT_EINVAL, "bad profile buffer");
  prof_drain();
  int32_t m = 0;
  for (int k = 0; k < kProfKinds && m < max_entries; ++k) {
    if (g_prof_n[k] == 0) continue;
    out[m].kind = k;
    out[m].launches = g_prof_n[k];
    out[m].total_ms = g_prof_ms[k];
    ++m;
  }
  return m;
}

size_t molt_sweep_workspace_bytes(const molt_grid* g, int32_t axis, int32_t precision, int64_t batch) {
  g_err.clear();
  if (check_grid(g, precision) != MOLT_OK || batch < 1 || (axis != 0 && axis != 1)) return 0;
  if (axis == 0 || g->ny == 1) return 256;
  const size_t esz = precision == MOLT_F64 ? 8 : 4;
  return al256(ypass_tot_elems(precision, g->ny, g->nx, (int)batch) * esz) + al256((size_t)2 * g->nx * batch * esz) +
         al256((size_t)g->nx * g->ny * batch * esz);
}

int32_t mol_t_helmholtz_sweep(const molt_grid* g, int32_t axis, double alpha, int32_t precision, const void* d_in,
                              void* d_out, int64_t batch, void* d_work, size_t work_bytes, void* stream) {
  g_err.clear();
  int32_t rc = sweep_check(g, axis, alpha, precision, d_in, d_out, batch);
  if (rc != MOLT_OK) return rc;
  if (axis == 0 || g->ny == 1) return sweep_impl(g, axis, alpha, precision, d_in, d_out, batch, nullptr, nullptr,
                                                 nullptr, (hipStream_t)stream);
  const size_t esz = precision == MOLT_F64 ? 8 : 4;
  const size_t need = molt_sweep_workspace_bytes(g, axis, precision, batch);
  if (!d_work || work_bytes < need) return fail(MOLT_EWORKSPACE, "workspace smaller than molt_sweep_workspace_bytes()");
  char* w = (char*)d_work;
  void* tot = w;
  void* jln = w + al256(ypass_tot_elems(precision, g->ny, g->nx, (int)batch) * esz);
  void* cpy = (char*)jln + al256((size_t)2 * g->nx * batch * esz);
  return sweep_impl(g, axis, alpha, precision, d_in, d_out, batch, tot, jln, cpy, (hipStream_t)stream);
}

size_t ch_workspace_bytes(const molt_grid* g, const molt_ch_params* p) {
  g_err.clear();
  if (check_params(p) != MOLT_OK || check_grid(g, p->precision) != MOLT_OK) return 0;
  return ch_layout(g, p->precision, ncomp_of(p), p->stepper == MOLT_BDF3).total;
}

int32_t ch_step(const molt_grid* g, const molt_ch_params* p, void* d_u, void* d_u_prev, void* d_work,
                size_t work_bytes, molt_step_info* info, void* stream) {
  g_err.clear();
  int32_t rc = check_params(p);
  if (rc != MOLT_OK) return rc;
  rc = check_grid(g, p->precision);
  if (rc != MOLT_OK) return rc;
  if (!d_u) return fail(MOLT_EINVAL, "d_u is NULL");
  if (p->stepper == MOLT_BDF3) {
    // d_u_prev: [u^{n-1} | u^{n-2}]; a BDF3 step with both, else an SDIRK2 step
    const size_t fb = (size_t)g->nx * g->ny * ncomp_of(p) * (p->precision == MOLT_F64 ? 8 : 4);
    void* prev2 = d_u_prev ? (char*)d_u_prev + fb : nullptr;
    if (p->have_prev >= 2 && d_u_prev)
      return step_impl(g, p, d_u, d_u_prev, true, d_work, work_bytes, info, (hipStream_t)stream, 0, 1.0, prev2);
    return sdirk2_impl(g, p, d_u, d_u_prev, prev2, d_work, work_bytes, info, (hipStream_t)stream);
  }
  const bool bdf2 = p->stepper == MOLT_BDF2 && p->have_prev && d_u_prev != nullptr;
  return step_impl(g, p, d_u, d_u_prev, bdf2, d_work, work_bytes, info, (hipStream_t)stream, 0);
}

int32_t ch_solve(const molt_grid* g, const molt_ch_params* p, void* d_u, int64_t nsteps, void* d_work,
                 size_t work_bytes, molt_step_info* per_step, void* stream) {
  g_err.clear();
  int32_t rc = check_params(p);
  if (rc != MOLT_OK) return rc;
  rc = check_grid(g, p->precision);
  if (rc != MOLT_OK) return rc;
  if (!d_u || nsteps < 0) return fail(MOLT_EINVAL, "d_u is NULL or nsteps < 0");
  const bool bdf3 = p->stepper == MOLT_BDF3;
  const Layout L = ch_layout(g, p->precision, ncomp_of(p), bdf3);
  if (!d_work || work_bytes < L.total) return fail(MOLT_EWORKSPACE, "workspace smaller than ch_workspace_bytes()");
  void* hist = (char*)d_work + L.fld[F_HIST];
  void* hist2 = (char*)d_work + L.fld[F_HIST2];
  int32_t status = MOLT_OK;
  int hint = 0;
  for (int64_t k = 0; k < nsteps; ++k) {
    const bool bdf2 = p->stepper == MOLT_BDF2 && k > 0;
    molt_step_info inf;
    if (bdf3 && k < 2)  // BDF3 start-up: two SDIRK2 steps (Sec. 4.4)
      rc = sdirk2_impl(g, p, d_u, hist, hist2, d_work, work_bytes, &inf, (hipStream_t)stream);
    else if (bdf3)
      rc = step_impl(g, p, d_u, hist, true, d_work, work_bytes, &inf, (hipStream_t)stream, hint, 1.0, hist2);
    else
      rc = step_impl(g, p, d_u, p->stepper == MOLT_BDF2 ? hist : nullptr, bdf2, d_work, work_bytes, &inf,
                     (hipStream_t)stream, hint);
    if (rc < 0) return rc;
    if (rc == MOLT_NOT_CONVERGED) status = MOLT_NOT_CONVERGED;
    hint = inf.iters;
    if (per_step) per_step[k] = inf;
  }
  return status;
}

int32_t molt_tune_get(int32_t precision, int32_t size_class, int32_t* kx, int32_t* ky) {
  g_err.clear();
  if ((precision != MOLT_F64 && precision != MOLT_F32) || size_class < 0 || size_class >= kTuneClasses || !kx || !ky)
    return fail(MOLT_EINVAL, "bad precision, size class or output pointer");
  int a, b;
  tune_get(precision, size_class, &a, &b);
  *kx = a;
  *ky = b;
  return MOLT_OK;
}

int32_t molt_tune_set(int32_t precision, int32_t size_class, int32_t kx, int32_t ky) {
  g_err.clear();
  if (!tune_valid(precision, size_class, kx, ky))
    return fail(MOLT_EINVAL, "shape not valid for this precision and size class");
  tune_set(precision, size_class, kx, ky);
  return MOLT_OK;
}

static size_t autotune_bytes(int prec, int n) {
  const size_t esz = prec == MOLT_F64 ? 8 : 4;
  return 7 * al256((size_t)n * n * esz) + al256(ypass_tot_elems(prec, n, n, 1) * esz) + al256((size_t)2 * n * esz);
}

size_t molt_autotune_workspace_bytes(int32_t precision, int32_t max_n) {
  g_err.clear();
  if ((precision != MOLT_F64 && precision != MOLT_F32) || max_n < 128 || max_n > xpass_max_n(precision)) return 0;
  return autotune_bytes(precision, max_n);
}

int32_t molt_autotune(int32_t precision, int32_t max_n, void* d_work, size_t work_bytes, void* stream) {
  g_err.clear();
  const size_t need = molt_autotune_workspace_bytes(precision, max_n);
  if (need == 0) return fail(MOLT_EINVAL, "precision or max_n out of range (128..8192 FP32, ..4096 FP64)");
  if (!d_work || work_bytes < need) return fail(MOLT_EWORKSPACE, "workspace smaller than molt_autotune_workspace_bytes()");
  hipStream_t s = (hipStream_t)stream;
  const bool prof = g_prof_on;
  g_prof_on = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int32_t rc = MOLT_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(MOLT_EHIP, "hipEventCreate");
  char* w = (char*)d_work;
  if (rc == MOLT_OK && launch_zero_ints((int*)w, (int)(need / 4), s) != hipSuccess)
    rc = fail(MOLT_EHIP, "workspace clear failed");
  const int reps = 8;
  // a candidate replaces the current entry only when it is faster by this
  // factor (launch-to-launch noise is a few percent; the table stays put on
  // a tie, so repeated tunings agree)
  const float margin = 0.97f;
  // average time of `reps` launches of fn (after one warm-up launch), ms
  auto timed = [&](auto fn) -> float {
    if (fn() != hipSuccess) return -1.0f;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r)
      if (fn() != hipSuccess) return -1.0f;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.0f;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0f;
    return ms / reps;
  };
  const size_t esz = precision == MOLT_F64 ? 8 : 4;
  for (int cls = 0; rc == MOLT_OK && cls <= tune_class(max_n); ++cls) {
    const int n = (128 << cls) < max_n ? (128 << cls) : max_n;
    const size_t fb = al256((size_t)n * n * esz);
    void* F[7];
    for (int f = 0; f < 7; ++f) F[f] = w + f * fb;
    void* tot = w + 7 * fb;
    void* jln = (char*)tot + al256(ypass_tot_elems(precision, n, n, 1) * esz);
    const LineCoef lc = make_line(n, MOLT_BC_PERIODIC, 4, 0.3 * n, 1.0 / n);  // nu = 0.3
    PassArgs a;
    memset(&a, 0, sizeof(a));
    a.sigma = 2.0;
    a.kappa = 0.5;
    a.mode = 1;
    int kx0, ky0;
    tune_get(precision, cls, &kx0, &ky0);
    int best_ky = ky0, best_kx = kx0;
    // the current entry first: it is the one to beat
    int kys[4] = {ky0, 4, 8, 16}, kxs[5] = {kx0, 4, 8, 16, 32};
    float best = -1.0f;
    for (int i = 0; i < 4; ++i) {
      const int ky = kys[i];
      if ((i > 0 && ky == ky0) || !tune_valid(precision, cls, kx0, ky)) continue;
      tune_set(precision, cls, kx0, ky);
      a.in[0] = F[0]; a.in[1] = F[1]; a.in[2] = F[2];
      a.out[0] = F[3]; a.out[1] = F[4];
      a.corr.seeds = nullptr;
      const float ms = timed([&] { return launch_ypass(precision, PROG_P1, lc, a, nullptr, n, 1, tot, jln, true, s); });
      if (ms < 0) { rc = fail(MOLT_EHIP, "autotune y-pass launch failed"); break; }
      if (best < 0 || ms < margin * best) { best = ms; best_ky = ky; }
    }
    best = -1.0f;
    for (int i = 0; rc == MOLT_OK && i < 5; ++i) {
      const int kx = kxs[i];
      if ((i > 0 && kx == kx0) || !tune_valid(precision, cls, kx, best_ky)) continue;
      tune_set(precision, cls, kx, best_ky);
      a.in[0] = F[0]; a.in[1] = F[1]; a.in[2] = F[2]; a.in[3] = F[3]; a.in[4] = F[4];
      a.out[0] = F[5]; a.out[1] = F[6];
      a.corr = make_ycorr(precision, lc, n, 2, tot);  // as after the deferred y-pass
      const float ms = timed([&] { return launch_xpass(precision, PROG_P2, lc, a, nullptr, n, nullptr, s); });
      if (ms < 0) { rc = fail(MOLT_EHIP, "autotune x-pass launch failed"); break; }
      if (best < 0 || ms < margin * best) { best = ms; best_kx = kx; }
    }
    tune_set(precision, cls, rc == MOLT_OK ? best_kx : kx0, rc == MOLT_OK ? best_ky : ky0);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  g_prof_on = prof;
  return rc;
}

size_t ch_batch_workspace_bytes(const molt_instance* inst, int32_t count) {
  g_err.clear();
  BatchPlan P;
  if (batch_plan(inst, count, P) != MOLT_OK) return 0;
  return P.total;
}

int32_t ch_solve_batch(const molt_instance* inst, int32_t count, void* d_work, size_t work_bytes,
                       molt_step_info* per_step, void* stream) {
  g_err.clear();
  return solve_batch_impl(inst, count, d_work, work_bytes, per_step, (hipStream_t)stream);
}

size_t ch_adaptive_workspace_bytes(const molt_grid* g, const molt_ch_params* p) {
  g_err.clear();
  if (check_adapt_params(p) != MOLT_OK || check_grid(g, p->precision) != MOLT_OK) return 0;
  return adapt_layout(g, p).total;
}

int32_t ch_solve_adaptive(const molt_grid* g, const molt_ch_params* p, const molt_adapt_params* ap, void* d_u,
                          void* d_work, size_t work_bytes, molt_adapt_record* rec, int32_t max_rec, int32_t* nrec,
                          double* t_final, void* stream) {
  g_err.clear();
  int32_t rc = check_adapt_params(p);
  if (rc != MOLT_OK) return rc;
  rc = check_grid(g, p->precision);
  if (rc != MOLT_OK) return rc;
  rc = check_adapt(ap);
  if (rc != MOLT_OK) return rc;
  if (!d_u || max_rec < 0) return fail(MOLT_EINVAL, "d_u is NULL or max_rec < 0");
  return solve_adaptive_impl(g, p, ap, d_u, d_work, work_bytes, rec, max_rec, nrec, t_final, (hipStream_t)stream);
}

size_t molt_server_footprint(const molt_instance* inst) {
  g_err.clear();
  if (!inst || check_instance(*inst, inst->params.precision) != MOLT_OK) return 0;
  return footprint(*inst, inst->params.precision);
}

size_t molt_server_bytes(int32_t precision, int32_t max_slots, size_t pool_bytes) {
  g_err.clear();
  if ((precision != MOLT_F64 && precision != MOLT_F32) || max_slots < 1 || max_slots > 65535 || pool_bytes == 0)
    return 0;
  return al256((size_t)max_slots * sizeof(SlotDesc)) + al256((size_t)max_slots * sizeof(SlotCtl)) +
         al256(server_map_cap(max_slots, pool_bytes) * sizeof(BlkMap)) + al256(pool_bytes);
}

int32_t molt_server_create(int32_t precision, int32_t max_slots, void* d_work, size_t work_bytes, void* stream,
                           molt_server** out) {
  g_err.clear();
  if (!out) return fail(MOLT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!stream) return fail(MOLT_EINVAL, "a server needs a non-default stream");
  const size_t fixed = molt_server_bytes(precision, max_slots, 256);
  if (fixed == 0) return fail(MOLT_EINVAL, "bad precision or max_slots");
  if (!d_work || work_bytes < fixed + 256) return fail(MOLT_EWORKSPACE, "workspace too small for a server");
  // pool = what is left after the descriptors, control words and maps
  size_t pool = work_bytes - fixed;
  while (pool > 256 && molt_server_bytes(precision, max_slots, pool) > work_bytes) pool -= 4096 < pool ? 4096 : 1;
  molt_server* S = new molt_server();
  S->prec = precision;
  S->max_slots = max_slots;
  S->s = (hipStream_t)stream;
  S->w = (char*)d_work;
  size_t off = 0;
  S->sd = (SlotDesc*)(S->w + off);
  off += al256((size_t)max_slots * sizeof(SlotDesc));
  S->ctl = (SlotCtl*)(S->w + off);
  off += al256((size_t)max_slots * sizeof(SlotCtl));
  S->map = (BlkMap*)(S->w + off);
  S->map_cap = server_map_cap(max_slots, pool);
  off += al256(S->map_cap * sizeof(BlkMap));
  S->pool_off = off;
  S->pool_end = work_bytes & ~(size_t)255;
  if (S->pool_end <= S->pool_off) {
    delete S;
    return fail(MOLT_EWORKSPACE, "workspace too small for a server");
  }
  S->free_[S->pool_off] = S->pool_end - S->pool_off;
  S->slots.resize(max_slots);
  S->insts.resize(max_slots);
  for (int i = max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
  std::vector<SlotCtl> idle(max_slots);
  for (SlotCtl& c : idle) c = SlotCtl{PH_IDLE, 0, 0, 0};
  hipError_t e = hipStreamCreateWithFlags(&S->cs, hipStreamNonBlocking);
  for (int b = 0; b < 2 && e == hipSuccess; ++b) {
    e = hipHostMalloc((void**)&S->pin[b], (size_t)max_slots * sizeof(SlotCtl), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev[b], hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->up_map[b], S->map_cap * sizeof(BlkMap), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_map[b], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(S->ev_map[b], S->s);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->up_desc, (size_t)max_slots * sizeof(SlotDesc), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->up_ctl, (size_t)max_slots * sizeof(SlotCtl), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemcpyAsync(S->ctl, idle.data(), idle.size() * sizeof(SlotCtl), hipMemcpyHostToDevice, S->s);
  if (e == hipSuccess) e = hipStreamSynchronize(S->s);
  if (e != hipSuccess) {
    molt_server_destroy(S);
    return fail(MOLT_EHIP, std::string("molt_server_create: ") + hipGetErrorString(e));
  }
  *out = S;
  return MOLT_OK;
}

int32_t molt_server_submit(molt_server* S, const molt_instance* inst, int64_t id) {
  g_err.clear();
  if (!S || !inst) return fail(MOLT_EINVAL, "NULL server or instance");
  const int32_t rc = check_instance(*inst, S->prec);
  if (rc != MOLT_OK) return rc;
  if (footprint(*inst, S->prec) > S->pool_end - S->pool_off || map_entries_max(*inst, S->prec) > S->map_cap)
    return fail(MOLT_EUNSUPPORTED, "the request does not fit this server's workspace");
  S->queue.push_back(molt_server::Req{id, *inst});
  return MOLT_OK;
}

int32_t molt_server_run(molt_server* S, int32_t rounds, int32_t* active, int32_t* queued) {
  g_err.clear();
  if (!S || rounds < 0) return fail(MOLT_EINVAL, "NULL server or negative rounds");
  const int32_t rc = server_run(S, rounds);
  if (active) *active = server_active(S);
  if (queued) *queued = (int32_t)S->queue.size();
  return rc;
}

int32_t molt_server_poll(molt_server* S, molt_result* out, int32_t max_results) {
  g_err.clear();
  if (!S || (!out && max_results > 0) || max_results < 0) return fail(MOLT_EINVAL, "bad poll arguments");
  int32_t m = 0;
  while (m < max_results && !S->done.empty()) {
    out[m++] = S->done.front();
    S->done.pop_front();
  }
  return m;
}

int32_t molt_server_destroy(molt_server* S) {
  g_err.clear();
  if (!S) return MOLT_OK;
  if (S->s) (void)hipStreamSynchronize(S->s);
  for (int b = 0; b < 2; ++b) {
    if (S->ev[b]) (void)hipEventDestroy(S->ev[b]);
    if (S->pin[b]) (void)hipHostFree(S->pin[b]);
    if (S->ev_map[b]) (void)hipEventDestroy(S->ev_map[b]);
    if (S->up_map[b]) (void)hipHostFree(S->up_map[b]);
  }
  if (S->up_desc) (void)hipHostFree(S->up_desc);
  if (S->up_ctl) (void)hipHostFree(S->up_ctl);
  if (S->cs) (void)hipStreamDestroy(S->cs);
  delete S;
  return MOLT_OK;
}

}  // extern "C"
