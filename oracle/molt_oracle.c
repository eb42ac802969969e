/*
 * molt_oracle.c -- FP64 CPU oracle of the MOL^T Cahn-Hilliard method
 * (Causley, Cho, Christlieb, "Method of lines transpose: energy gradient flows
 * using direct operator inversion for phase field models", arXiv:1611.04214).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * Everything is FP64.  Each function cites the passage of the paper it follows.
 * Where the paper is silent or has a typo, the reading taken is stated at the
 * function; the same readings are listed in the design notes of the repository.
 *
 * Layout: a 2D field is row-major, f[iy*nx + ix]; rows are x-lines, columns
 * are y-lines.  ny == 1 is a 1D problem (no y-direction operator at all).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#define OR_BC_PERIODIC 0
#define OR_BC_NEUMANN 1
#define OR_BC_DIRICHLET 2

#define OR_BE 0
#define OR_BDF2 1
#define OR_BDF3 2

#define OR_INIT_PREV 0
#define OR_INIT_LINEAR 1

#define OR_MAXM 6

/* ------------------------------------------------------------------------ */
/* Problem description (mirrors the paper's statement of the problem:       */
/* grid and domain, boundary type, quadrature order M, eps, dt, stepper).   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int nx, ny;          /* periodic: unique nodes per line; Neumann: nodes incl. both ends */
  double x0, x1, y0, y1;
  int bc;              /* OR_BC_* */
  int M;               /* quadrature order: 2, 4 or 6 */
} or_grid;

typedef struct {
  double eps, dt, tol;
  double sigma0;       /* f'(0) in the shifted variable: 2 for CH */
  int stepper;         /* OR_BE or OR_BDF2 */
  int max_iter;
  int init;            /* OR_INIT_PREV (v^{n+1,0} = v^n) or OR_INIT_LINEAR (v^{n+1,0} = R) */
  int fixed_iters;     /* >0: run exactly this many iterations (parity mode) */
  int reaction;        /* 0: Cahn-Hilliard f(v) = v^3 - 3v^2 + 2v; 1: linear f(v) = react_k*v (test hook);
                          2: the vector model's reaction on the real axis, f(v) = 6((v-1)^5 - (v-1)^2)
                          (test hook) */
  double react_k;
  double omega;        /* BDF2 step ratio dt_n / dt_{n-1}; 0 or 1: constant steps */
} or_params;

typedef struct {
  int iters;
  double residual;     /* last max-norm increment */
  double mass, energy; /* of u^{n+1} (vector model: mass of the first component) */
  double s1, s2, sigma;
  double mass2;        /* vector model: mass of the second component */
} or_info;

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1] (Newton iteration on the Legendre           */
/* recurrence).  Used to integrate exp(-nu s) times a Lagrange polynomial.   */
/* ------------------------------------------------------------------------ */
static void gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < n; i++) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double p0 = 0, p1 = 0, dp = 1;
    for (int it = 0; it < 200; it++) {
      p0 = 1.0;
      p1 = z;
      for (int k = 2; k <= n; k++) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-17) break;
    }
    p0 = 1.0;
    p1 = z;
    for (int k = 2; k <= n; k++) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* Lagrange basis polynomial i on the integer nodes 0..M, evaluated at t. */
static double lagrange(int M, int i, double t) {
  double p = 1.0;
  for (int k = 0; k <= M; k++)
    if (k != i) p *= (t - k) / (double)(i - k);
  return p;
}

/*
 * Local quadrature weights of Sec. 3.2 (eqs. IL, IR and the M=2 weights P,Q,R
 * that follow them).  The local integral over one cell, with the kernel
 * alpha*exp(-alpha*|x_j - x'|) (no factor 1/2: see line_inverse), is
 *     nu * int_0^1 exp(-nu*s) p(x_j -+ s*h) ds,
 * where p is the degree-M Lagrange interpolant of v on M+1 consecutive nodes.
 * The paper prints only M=2 (nodes j-1, j, j+1) and says higher-order weights
 * are precomputed.  Reading: the window of M+1 nodes is centred on node j
 * (the node at which the recursion is evaluated), shifted to the nearest
 * in-range window near a non-periodic end.
 *
 * wl[r][i]: weight of window node i for the cell LEFT of the node at window
 *           position r (i.e. the cell [x_{j-1}, x_j] of J^L_j, with j = lo + r);
 * wr[r][i]: same for the cell RIGHT of it ([x_j, x_{j+1}] of J^R_j).
 * Computed by composite Gauss-Legendre quadrature (8 panels x 16 points).
 */
typedef struct {
  int M;
  double nu, d;
  double wl[OR_MAXM + 1][OR_MAXM + 1];
  double wr[OR_MAXM + 1][OR_MAXM + 1];
} or_weights;

static void make_weights(int M, double nu, or_weights *W) {
  enum { NP = 16, NPAN = 8 };
  double gx[NP], gw[NP];
  gauss_legendre(NP, gx, gw);
  memset(W, 0, sizeof(*W));
  W->M = M;
  W->nu = nu;
  W->d = exp(-nu);
  for (int r = 0; r <= M; r++) {
    for (int i = 0; i <= M; i++) {
      double sl = 0.0, sr = 0.0;
      for (int pan = 0; pan < NPAN; pan++) {
        double a = (double)pan / NPAN, b = (double)(pan + 1) / NPAN;
        for (int q = 0; q < NP; q++) {
          double s = 0.5 * (b - a) * gx[q] + 0.5 * (a + b);
          double ws = 0.5 * (b - a) * gw[q] * nu * exp(-nu * s);
          sl += ws * lagrange(M, i, r - s);
          sr += ws * lagrange(M, i, r + s);
        }
      }
      W->wl[r][i] = sl;
      W->wr[r][i] = sr;
    }
  }
}

/* Small cache of weight tables keyed by (M, nu): the tables depend only on
 * them, and a time step applies the same few operators many times.  Filled
 * and read on the calling thread only. */
#define OR_WCACHE 8
static or_weights or_wcache[OR_WCACHE];
static int or_wcache_n = 0, or_wcache_next = 0;

static const or_weights *get_weights(int M, double nu) {
  for (int i = 0; i < or_wcache_n; i++)
    if (or_wcache[i].M == M && or_wcache[i].nu == nu) return &or_wcache[i];
  int slot = or_wcache_next;
  make_weights(M, nu, &or_wcache[slot]);
  or_wcache_next = (or_wcache_next + 1) % OR_WCACHE;
  if (or_wcache_n < OR_WCACHE) or_wcache_n++;
  return &or_wcache[slot];
}

/* M=2 weights exactly as printed after eqs. IL/IR (Sec. 3.2).  Exposed for
 * the pin that the general construction reproduces them. */
void oracle_pqr(double nu, double *P, double *Q, double *R) {
  double d = exp(-nu);
  *P = 1.0 - (1.0 - d) / nu;
  *Q = -d + (1.0 - d) / nu;
  *R = (1.0 - d) / (nu * nu) - (1.0 + d) / (2.0 * nu);
}

/* Expose the cell weights (interior, centred window) for tests. */
int oracle_weights(int M, double nu, double *wl_centre, double *wr_centre) {
  if (M < 2 || M > OR_MAXM || (M & 1) || !(nu > 0)) return -1;
  or_weights W;
  make_weights(M, nu, &W);
  for (int i = 0; i <= M; i++) {
    wl_centre[i] = W.wl[M / 2][i];
    wr_centre[i] = W.wr[M / 2][i];
  }
  return 0;
}

/* Exposed for tests: weights for any window position r. */
int oracle_weights_window(int M, double nu, int r, double *wl, double *wr) {
  if (M < 2 || M > OR_MAXM || (M & 1) || !(nu > 0) || r < 0 || r > M) return -1;
  or_weights W;
  make_weights(M, nu, &W);
  for (int i = 0; i <= M; i++) {
    wl[i] = W.wl[r][i];
    wr[i] = W.wr[r][i];
  }
  return 0;
}

/*
 * One line of L^{-1} = (I - d_xx/alpha^2)^{-1}, Sec. 3.1-3.2:
 *   L^{-1}[v](x) = I[v](x) + B_a exp(-alpha(x-a)) + B_b exp(-alpha(b-x)),
 *   I[v](x) = (alpha/2) int_a^b exp(-alpha|x-x'|) v(x') dx'   (eq. Iu),
 * with I split into left and right parts computed by the exact exponential
 * recursions (eqs. IL, IR).  The printed weights carry the kernel alpha*exp
 * (P+Q = 1-d), so the sweeps below accumulate 2*I^L and 2*I^R and the
 * particular solution is I_j = (IL~_j + IR~_j)/2.  Reading: the factor 1/2 of
 * eq. Iu is applied here (it makes L^{-1}[1] = 1).
 *
 * Periodic (eq. homogeneous): B_a = I_N/(1-mu), B_b = I_0/(1-mu), mu = d^N,
 *   n unique nodes, N = n cells, v_N = v_0 and the stencil wraps.
 * Neumann (the "analogous 2x2 system" the paper mentions, derived from
 *   w'(a) = w'(b) = 0 with I'(a) = alpha*I_0, I'(b) = -alpha*I_N):
 *   B_a = (I_0 + mu I_N)/(1-mu^2), B_b = (I_N + mu I_0)/(1-mu^2),
 *   n nodes including both ends, N = n-1 cells.
 * Dirichlet (w(a) = w(b) = 0):
 *   B_a = (mu I_N - I_0)/(1-mu^2), B_b = (mu I_0 - I_N)/(1-mu^2).
 *
 * in and out may not alias.  tmpL, tmpR: scratch of n+1 doubles.
 */
static void line_inverse(int bc, const or_weights *W, int n, const double *v, double *w,
                         double *IL, double *IR) {
  const int M = W->M, h2 = M / 2;
  const double d = W->d, nu = W->nu;
  const int N = (bc == OR_BC_PERIODIC) ? n : n - 1; /* number of cells */
#define VAL(k) (bc == OR_BC_PERIODIC ? v[(((k) % n) + n) % n] : v[(k)])
  /* left-to-right recursion (eq. IL) */
  IL[0] = 0.0;
  for (int j = 1; j <= N; j++) {
    int lo = j - h2;
    if (bc != OR_BC_PERIODIC) {
      if (lo < 0) lo = 0;
      if (lo > N - M) lo = N - M;
    }
    int r = j - lo;
    double J = 0.0;
    for (int i = 0; i <= M; i++) J += W->wl[r][i] * VAL(lo + i);
    IL[j] = d * IL[j - 1] + J;
  }
  /* right-to-left recursion (eq. IR) */
  IR[N] = 0.0;
  for (int j = N - 1; j >= 0; j--) {
    int lo = j - h2;
    if (bc != OR_BC_PERIODIC) {
      if (lo < 0) lo = 0;
      if (lo > N - M) lo = N - M;
    }
    int r = j - lo;
    double J = 0.0;
    for (int i = 0; i <= M; i++) J += W->wr[r][i] * VAL(lo + i);
    IR[j] = d * IR[j + 1] + J;
  }
#undef VAL
  double I0 = 0.5 * (IL[0] + IR[0]);
  double IN = 0.5 * (IL[N] + IR[N]);
  double mu = exp(-nu * N);
  double Ba, Bb;
  if (bc == OR_BC_PERIODIC) {
    Ba = IN / (1.0 - mu);
    Bb = I0 / (1.0 - mu);
  } else if (bc == OR_BC_NEUMANN) {
    Ba = (I0 + mu * IN) / (1.0 - mu * mu);
    Bb = (IN + mu * I0) / (1.0 - mu * mu);
  } else {
    Ba = (mu * IN - I0) / (1.0 - mu * mu);
    Bb = (mu * I0 - IN) / (1.0 - mu * mu);
  }
  for (int j = 0; j < n; j++) {
    double Ij = 0.5 * (IL[j] + IR[j]);
    w[j] = Ij + Ba * exp(-nu * j) + Bb * exp(-nu * (N - j));
  }
}

/* Grid spacing along one axis. */
static double spacing(int bc, int n, double a, double b) {
  return (bc == OR_BC_PERIODIC) ? (b - a) / n : (b - a) / (n - 1);
}

static int grid_ok(const or_grid *g) {
  if (!g || g->nx < 1 || g->ny < 1) return 0;
  if (g->M < 2 || g->M > OR_MAXM || (g->M & 1)) return 0;
  if (g->bc < 0 || g->bc > 2) return 0;
  if (g->nx < g->M + 1) return 0;
  if (g->ny != 1 && g->ny < g->M + 1) return 0;
  if (!(g->x1 > g->x0)) return 0;
  if (g->ny > 1 && !(g->y1 > g->y0)) return 0;
  return 1;
}

/* Apply the line inverse with parameter alpha along x (every row) or y (every
 * column) of the field.  ny == 1 and axis y: the identity (1D problem). */
static void sweep(const or_grid *g, int axis, double alpha, const double *in, double *out) {
  const int nx = g->nx, ny = g->ny;
  if (axis == 1 && ny == 1) {
    if (out != in) memcpy(out, in, sizeof(double) * (size_t)nx);
    return;
  }
  const int n = axis == 0 ? nx : ny;
  const double h = axis == 0 ? spacing(g->bc, nx, g->x0, g->x1) : spacing(g->bc, ny, g->y0, g->y1);
  const or_weights *W = get_weights(g->M, alpha * h);
  const int nlines = axis == 0 ? ny : nx;
#pragma omp parallel if (nlines > 1)
  {
    double *line = (double *)malloc(sizeof(double) * (size_t)n);
    double *res = (double *)malloc(sizeof(double) * (size_t)n);
    double *IL = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *IR = (double *)malloc(sizeof(double) * (size_t)(n + 1));
#pragma omp for schedule(static)
    for (int l = 0; l < nlines; l++) {
      for (int k = 0; k < n; k++) line[k] = axis == 0 ? in[(size_t)l * nx + k] : in[(size_t)k * nx + l];
      line_inverse(g->bc, W, n, line, res, IL, IR);
      for (int k = 0; k < n; k++) {
        if (axis == 0)
          out[(size_t)l * nx + k] = res[k];
        else
          out[(size_t)k * nx + l] = res[k];
      }
    }
    free(line);
    free(res);
    free(IL);
    free(IR);
  }
}

/* Public: one directional sweep of L^{-1} over a 2D (or 1D) field. */
int oracle_sweep(const or_grid *g, int axis, double alpha, const double *in, double *out) {
  if (!grid_ok(g) || (axis != 0 && axis != 1) || !(alpha > 0)) return -1;
  sweep(g, axis, alpha, in, out);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Stepper algebra, Sec. 3.1 (eqs. CH_BE_fixed2_factor, CH_BE_fixed_complete) */
/* and Sec. 4.1 (BDF2 factorizations).                                       */
/*                                                                          */
/* The scheme for v^{n+1} is (I - a*d_xx(f) + a*eps^2 d_xxxx) v = rhs with   */
/* a = beta*dt (beta = 1 for BE, 2/3 for BDF2).  Writing f(v) = sigma*v +    */
/* g(v) and moving a*Lap(g) to the right-hand side, the left operator        */
/* I - sigma*a*Lap + a*eps^2*Lap^2 factors as (I - s1 Lap)(I - s2 Lap):      */
/*  - factorization regime (sigma0*a/2)^2 >= a*eps^2: sigma = sigma0,         */
/*    s1,2 = sigma0*a/2 +- sqrt((sigma0*a/2)^2 - a*eps^2)  (for sigma0 = 2:   */
/*    a +- sqrt(a^2 - a*eps^2), the paper's 1/alpha_{1,2}^2);                 */
/*  - completed-square regime otherwise: s1 = s2 = sqrt(eps^2 a)              */
/*    (the paper's 1/alpha^2) and sigma = 2*sqrt(eps^2/a), which is the       */
/*    lagged term f - 2 sqrt(eps^2/dt) v of Sec. 4.1 (Sec. 3.1 prints        */
/*    2(1+sqrt(eps^2/dt)) with f~ = f - 2v; reading: the same term).         */
/* s2 is taken as a*eps^2/s1 (the product of the two roots), which avoids    */
/* the cancellation of the minus root.                                        */
/* ------------------------------------------------------------------------ */
static void stepper_params(double eps, double a, double sigma0, double *s1, double *s2, double *sigma) {
  double half = 0.5 * sigma0 * a;
  if (half * half >= a * eps * eps) {
    *sigma = sigma0;
    *s1 = half + sqrt(half * half - a * eps * eps);
    *s2 = a * eps * eps / *s1;
  } else {
    *sigma = 2.0 * sqrt(eps * eps / a);
    *s1 = sqrt(eps * eps * a);
    *s2 = *s1;
  }
}

int oracle_stepper_params(double eps, double dt, int stepper, int first, double sigma0, double *out3) {
  double beta = first ? 1.0 : (stepper == OR_BDF2 ? 2.0 / 3.0 : (stepper == OR_BDF3 ? 6.0 / 11.0 : 1.0));
  stepper_params(eps, beta * dt, sigma0, &out3[0], &out3[1], &out3[2]);
  return 0;
}

/* Reaction in the shifted variable v = u+1 (eq. CahnHilliard_v):
 * f(v) = v^3 - 3v^2 + 2v. */
static double f_react(double v) { return v * v * v - 3.0 * v * v + 2.0 * v; }

/* ------------------------------------------------------------------------ */
/* Diagnostics (reading: the paper has no discrete energy).                  */
/* Energy of eq. EnergyFunctional with forward differences and, for the      */
/* non-periodic ends, trapezoid weights; mass = integral of u by the same    */
/* rule.                                                                     */
/* ------------------------------------------------------------------------ */
static double tw(int bc, int k, int n) {
  if (bc == OR_BC_PERIODIC) return 1.0;
  return (k == 0 || k == n - 1) ? 0.5 : 1.0;
}

double oracle_mass(const or_grid *g, const double *u) {
  const int nx = g->nx, ny = g->ny;
  double hx = spacing(g->bc, nx, g->x0, g->x1);
  double hy = ny > 1 ? spacing(g->bc, ny, g->y0, g->y1) : 1.0;
  double s = 0.0;
  for (int iy = 0; iy < ny; iy++)
    for (int ix = 0; ix < nx; ix++)
      s += tw(g->bc, ix, nx) * (ny > 1 ? tw(g->bc, iy, ny) : 1.0) * u[(size_t)iy * nx + ix];
  return s * hx * hy;
}

double oracle_energy(const or_grid *g, double eps, const double *u) {
  const int nx = g->nx, ny = g->ny;
  const int per = g->bc == OR_BC_PERIODIC;
  double hx = spacing(g->bc, nx, g->x0, g->x1);
  double hy = ny > 1 ? spacing(g->bc, ny, g->y0, g->y1) : 1.0;
  double e = 0.0;
  for (int iy = 0; iy < ny; iy++) {
    double wy = ny > 1 ? tw(g->bc, iy, ny) : 1.0;
    for (int ix = 0; ix < nx; ix++) {
      double wx = tw(g->bc, ix, nx);
      double uu = u[(size_t)iy * nx + ix];
      double F = 0.25 * (uu * uu - 1.0) * (uu * uu - 1.0);
      e += wx * wy * F * hx * hy;
      /* x edge to the right of this node */
      if (per || ix < nx - 1) {
        double un = u[(size_t)iy * nx + (ix + 1) % nx];
        double gx = (un - uu) / hx;
        e += 0.5 * eps * eps * gx * gx * wy * hx * hy;
      }
      if (ny > 1 && (per || iy < ny - 1)) {
        double un = u[(size_t)((iy + 1) % ny) * nx + ix];
        double gy = (un - uu) / hy;
        e += 0.5 * eps * eps * gy * gy * wx * hx * hy;
      }
    }
  }
  return e;
}

/* ------------------------------------------------------------------------ */
/* One time step, Sec. 5.1 (eqs. CH_BE_2D_3, CH_2D_Doperator1/2) written    */
/* for two possibly different factors (reading: the paper writes the 2D     */
/* iteration for the completed square only and says the other cases follow */
/* "similarly"; with A_i = Lx_i Ly_i and D_i = (I - Lx_i^{-1})(I - Ly_i^{-1})*/
/* the lagged splitting error of (A_1 - E_1)(A_2 - E_2) gives                */
/*   v^{k+1} = A1^{-1} A2^{-1} rhs + (a/s1) A2^{-1} C1 g(v^k)                */
/*             + D1 v^k + D2 (v^k - D1 v^k),  C1 = A1^{-1} - I + D1,          */
/* which for s1 = s2 is the paper's (LxLy)^{-2} v^n + (LxLy)^{-1} C1[..]     */
/* + C2 v^k with C2 = 2D - D^2).  The factor a/s1 is alpha_1^2 * a of the    */
/* remark on L^{-1} d_xx = alpha^2 (L^{-1} - I), peeled with the smaller      */
/* alpha (reading).                                                          */
/* In 1D (ny == 1) Ly^{-1} = I, so D_i = 0 and this is                       */
/*   v^{k+1} = L1^{-1} L2^{-1} rhs + (a/s1) L2^{-1}(L1^{-1} - I) g(v^k).      */
/* rhs = v^n (BE, eq. CH_BE) or (4v^n - v^{n-1})/3 (BDF2, eq. BDF2).         */
/* Stop when max|v^{k+1}-v^k| < tol or k = max_iter (Sec. 4.4), or after     */
/* exactly fixed_iters iterations.                                           */
/* u and u_prev hold u = v - 1 (the paper's variable); u_prev == NULL or    */
/* stepper == BE gives a BE step.  On return u holds u^{n+1}; u_prev is not   */
/* modified (the caller rotates history).                                    */
/* ------------------------------------------------------------------------ */
static void Ainv(const or_grid *g, double alpha, const double *in, double *out, double *tmp) {
  sweep(g, 1, alpha, in, tmp);   /* Ly^{-1} */
  sweep(g, 0, alpha, tmp, out);  /* Lx^{-1} */
}

/* D w = (I - Lx^{-1})(I - Ly^{-1}) w */
static void Dop(const or_grid *g, double alpha, const double *in, double *out, double *t1, size_t n) {
  sweep(g, 1, alpha, in, t1);
  for (size_t i = 0; i < n; i++) t1[i] = in[i] - t1[i];  /* (I - Ly^{-1}) w */
  sweep(g, 0, alpha, t1, out);
  for (size_t i = 0; i < n; i++) out[i] = t1[i] - out[i]; /* (I - Lx^{-1}) (...) */
}

/* u_prev2 != NULL (with u_prev) and stepper == OR_BDF3: a BDF3 step (eq. BDF3),
 * (I - beta dt F) v^{n+1} = (18 v^n - 9 v^{n-1} + 2 v^{n-2})/11, beta = 6/11. */
static int step_core(const or_grid *g, const or_params *p, double *u, const double *u_prev,
                     const double *u_prev2, or_info *info) {
  if (!grid_ok(g) || !p || !u) return -1;
  if (!(p->eps > 0) || !(p->dt > 0) || !(p->sigma0 > 0)) return -1;
  const size_t n = (size_t)g->nx * g->ny;
  const int bdf3 = (p->stepper == OR_BDF3) && u_prev != NULL && u_prev2 != NULL;
  const int bdf2 = !bdf3 && (p->stepper == OR_BDF2) && u_prev != NULL;
  /* variable-step BDF2 (reading; the paper writes constant steps): with
   * w = dt_n/dt_{n-1}, ((1+2w)/(1+w)) v^{n+1} - (1+w) v^n + (w^2/(1+w)) v^{n-1}
   * = dt_n F(v^{n+1}), i.e. v^{n+1} - beta dt_n F = rc0 v^n + rc1 v^{n-1} with
   * beta = (1+w)/(1+2w), rc0 = (1+w)^2/(1+2w), rc1 = -w^2/(1+2w); w = 1 gives
   * 2/3, 4/3, -1/3 (eq. BDF2). */
  const double w = (p->omega > 0.0) ? p->omega : 1.0;
  const double beta = bdf3 ? 6.0 / 11.0 : (bdf2 ? (1.0 + w) / (1.0 + 2.0 * w) : 1.0);
  const double rc0 = (1.0 + w) * (1.0 + w) / (1.0 + 2.0 * w), rc1 = -w * w / (1.0 + 2.0 * w);
  const double a = beta * p->dt;
  double s1, s2, sigma;
  stepper_params(p->eps, a, p->sigma0, &s1, &s2, &sigma);
  const double al1 = 1.0 / sqrt(s1), al2 = 1.0 / sqrt(s2);

  double *vn = (double *)malloc(sizeof(double) * n);
  double *rhs = (double *)malloc(sizeof(double) * n);
  double *R = (double *)malloc(sizeof(double) * n);
  double *v = (double *)malloc(sizeof(double) * n);
  double *gk = (double *)malloc(sizeof(double) * n);
  double *c1 = (double *)malloc(sizeof(double) * n);
  double *t1 = (double *)malloc(sizeof(double) * n);
  double *t2 = (double *)malloc(sizeof(double) * n);
  double *dv = (double *)malloc(sizeof(double) * n);
  double *q = (double *)malloc(sizeof(double) * n);
  double *vnew = (double *)malloc(sizeof(double) * n);
  if (!vn || !rhs || !R || !v || !gk || !c1 || !t1 || !t2 || !dv || !q || !vnew) return -2;

  for (size_t i = 0; i < n; i++) vn[i] = u[i] + 1.0;
  if (bdf3)
    for (size_t i = 0; i < n; i++)
      rhs[i] = (18.0 * vn[i] - 9.0 * (u_prev[i] + 1.0) + 2.0 * (u_prev2[i] + 1.0)) / 11.0;
  else if (bdf2 && w == 1.0)
    for (size_t i = 0; i < n; i++) rhs[i] = (4.0 * vn[i] - (u_prev[i] + 1.0)) / 3.0;
  else if (bdf2)
    for (size_t i = 0; i < n; i++) rhs[i] = rc0 * vn[i] + rc1 * (u_prev[i] + 1.0);
  else
    memcpy(rhs, vn, sizeof(double) * n);

  /* R = A1^{-1} A2^{-1} rhs */
  Ainv(g, al2, rhs, t2, t1);
  Ainv(g, al1, t2, R, t1);

  if (p->init == OR_INIT_LINEAR)
    memcpy(v, R, sizeof(double) * n);
  else
    memcpy(v, vn, sizeof(double) * n);

  const double kappa = a / s1;
  int k = 0;
  double res = 0.0;
  for (;;) {
    /* g(v^k) = f(v^k) - sigma v^k */
    for (size_t i = 0; i < n; i++) {
      double f;
      if (p->reaction == 1) {
        f = p->react_k * v[i];
      } else if (p->reaction == 2) {
        const double x = v[i] - 1.0;
        f = 6.0 * (x * x * x * x * x - x * x);
      } else {
        f = f_react(v[i]);
      }
      gk[i] = f - sigma * v[i];
    }
    /* C1 g = A1^{-1} g - g + D1 g */
    Ainv(g, al1, gk, c1, t1);
    Dop(g, al1, gk, t2, t1, n);
    for (size_t i = 0; i < n; i++) c1[i] = c1[i] - gk[i] + t2[i];
    /* A2^{-1} C1 g */
    Ainv(g, al2, c1, t2, t1);
    /* D1 v and D2 (v - D1 v) */
    Dop(g, al1, v, dv, t1, n);
    for (size_t i = 0; i < n; i++) q[i] = v[i] - dv[i];
    Dop(g, al2, q, c1, t1, n);
    res = 0.0;
    for (size_t i = 0; i < n; i++) {
      vnew[i] = R[i] + kappa * t2[i] + dv[i] + c1[i];
      double e = fabs(vnew[i] - v[i]);
      if (e > res) res = e;
    }
    memcpy(v, vnew, sizeof(double) * n);
    k++;
    if (p->fixed_iters > 0) {
      if (k >= p->fixed_iters) break;
    } else if (res < p->tol || k >= p->max_iter) {
      break;
    }
  }
  for (size_t i = 0; i < n; i++) u[i] = v[i] - 1.0;
  if (info) {
    info->iters = k;
    info->residual = res;
    info->mass = oracle_mass(g, u);
    info->energy = oracle_energy(g, p->eps, u);
    info->s1 = s1;
    info->s2 = s2;
    info->sigma = sigma;
    info->mass2 = 0.0;
  }
  free(vn); free(rhs); free(R); free(v); free(gk); free(c1);
  free(t1); free(t2); free(dv); free(q); free(vnew);
  return (p->fixed_iters <= 0 && res >= p->tol) ? 1 : 0;
}

int oracle_step(const or_grid *g, const or_params *p, double *u, const double *u_prev, or_info *info) {
  return step_core(g, p, u, u_prev, NULL, info);
}

int oracle_bdf3_step(const or_grid *g, const or_params *p, double *u, const double *u_prev,
                     const double *u_prev2, or_info *info) {
  if (!u_prev || !u_prev2 || p->stepper != OR_BDF3) return -1;
  return step_core(g, p, u, u_prev, u_prev2, info);
}

/* SDIRK2 (Sec. 4.2, eta = 1 - sqrt(2)/2).  With the stage values
 * V1 = v^n + eta dt K1 and V2 = W + eta dt K2, W = v^n + (1-eta) dt K1, the two
 * stage equations read (I + eta eps^2 dt d4) V1 = v^n + eta dt d2 f(V1) and
 * (I + eta eps^2 dt d4) V2 = W + eta dt d2 f(V2), i.e. two BE steps of size
 * eta dt (from v^n, then from W = v^n + ((1-eta)/eta)(V1 - v^n)), and
 * v^{n+1} = V2.  (Reading: the stages are solved in this form; the fixed
 * points are the paper's stage solutions.)  info: the second stage's report,
 * iters = both stages' iterations. */
int oracle_sdirk2_step(const or_grid *g, const or_params *p, double *u, or_info *info) {
  const size_t n = (size_t)g->nx * g->ny;
  const double eta = 1.0 - sqrt(2.0) / 2.0;
  or_params q = *p;
  q.stepper = OR_BE;
  q.dt = eta * p->dt;
  double *v1 = (double *)malloc(sizeof(double) * n);
  if (!v1) return -2;
  memcpy(v1, u, sizeof(double) * n);
  or_info i1;
  int rc1 = step_core(g, &q, v1, NULL, NULL, &i1);
  if (rc1 < 0) { free(v1); return rc1; }
  for (size_t i = 0; i < n; i++) u[i] = u[i] + (1.0 - eta) / eta * (v1[i] - u[i]);  /* W */
  int rc2 = step_core(g, &q, u, NULL, NULL, info);
  free(v1);
  if (rc2 < 0) return rc2;
  if (info) info->iters += i1.iters;
  return (rc1 > 0 || rc2 > 0) ? 1 : 0;
}

/* nsteps steps; BDF2 takes a BE first step (reading: the paper's start-up
 * for BDF2 is not stated; a BE first step reproduces its Table 1); BDF3 takes
 * two SDIRK2 steps first (Sec. 4.4).
 * infos: nsteps entries or NULL.  Returns 1 if any step hit max_iter. */
int oracle_solve(const or_grid *g, const or_params *p, double *u, int nsteps, or_info *infos) {
  if (!grid_ok(g) || !p || !u || nsteps < 0) return -1;
  const size_t n = (size_t)g->nx * g->ny;
  double *prev = (double *)malloc(sizeof(double) * n);
  double *prev2 = (double *)malloc(sizeof(double) * n);
  double *cur = (double *)malloc(sizeof(double) * n);
  int status = 0;
  for (int s = 0; s < nsteps; s++) {
    memcpy(cur, u, sizeof(double) * n);
    int rc;
    if (p->stepper == OR_BDF3)
      rc = s < 2 ? oracle_sdirk2_step(g, p, u, infos ? &infos[s] : NULL)
                 : step_core(g, p, u, prev, prev2, infos ? &infos[s] : NULL);
    else
      rc = step_core(g, p, u, s == 0 ? NULL : prev, NULL, infos ? &infos[s] : NULL);
    if (rc < 0) { status = rc; break; }
    if (rc > 0) status = 1;
    memcpy(prev2, prev, sizeof(double) * n);
    memcpy(prev, cur, sizeof(double) * n);
  }
  free(prev);
  free(prev2);
  free(cur);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Vector Cahn-Hilliard (Sec. 2 eqs. CH_vector, CH_vector_reaction; Sec. 5.2 */
/* eqs. CH_vector_linearize, CH_vector_BE, CH_vector_fixed1/2).              */
/* u = (u1, u2); W(u) = prod_{i=1..3} |u - z_i|^2 with z_i the cube roots of */
/* unity in the (u1,u2) plane.  The scheme shifts by z_3 = (-1/2,-sqrt3/2): */
/* v = u - z_3, and applies the scalar machinery to each component with the  */
/* reaction g_c(v) = dW/du_c(v + z_3) - sigma v_c and sigma0 = 18 (the       */
/* Hessian of W at its minima, eq. Jacobian); the two factorizations of      */
/* eqs. CH_vector_fixed1/2 are the unified stepper with sigma0 = 18.         */
/* A vector field is stored component-major: u[0..n) = u1, u[n..2n) = u2.    */
/* ------------------------------------------------------------------------ */
static const double OR_Z[3][2] = {{1.0, 0.0},
                                  {-0.5, 0.86602540378443864676372317075294},
                                  {-0.5, -0.86602540378443864676372317075294}};

/* W from its definition: the product of the three squared distances. */
double oracle_vch_W(double u1, double u2) {
  double w = 1.0;
  for (int i = 0; i < 3; i++) {
    const double a = u1 - OR_Z[i][0], b = u2 - OR_Z[i][1];
    w *= a * a + b * b;
  }
  return w;
}

/* grad W by the product rule: dW/du_c = sum_i 2 (u_c - z_{i,c}) prod_{j != i} d_j. */
void oracle_vch_gradW(double u1, double u2, double *g) {
  double d[3];
  for (int i = 0; i < 3; i++) {
    const double a = u1 - OR_Z[i][0], b = u2 - OR_Z[i][1];
    d[i] = a * a + b * b;
  }
  g[0] = g[1] = 0.0;
  for (int i = 0; i < 3; i++) {
    const double others = d[(i + 1) % 3] * d[(i + 2) % 3];
    g[0] += 2.0 * (u1 - OR_Z[i][0]) * others;
    g[1] += 2.0 * (u2 - OR_Z[i][1]) * others;
  }
}

/* Energy of eq. EnergyFunctional_vector with the discretization of
 * oracle_energy (forward differences, trapezoid weights off the periodic case). */
double oracle_vch_energy(const or_grid *g, double eps, const double *u) {
  const int nx = g->nx, ny = g->ny;
  const size_t n = (size_t)nx * ny;
  const int per = g->bc == OR_BC_PERIODIC;
  double hx = spacing(g->bc, nx, g->x0, g->x1);
  double hy = ny > 1 ? spacing(g->bc, ny, g->y0, g->y1) : 1.0;
  double e = 0.0;
  for (int iy = 0; iy < ny; iy++) {
    double wy = ny > 1 ? tw(g->bc, iy, ny) : 1.0;
    for (int ix = 0; ix < nx; ix++) {
      double wx = tw(g->bc, ix, nx);
      const size_t i = (size_t)iy * nx + ix;
      e += wx * wy * oracle_vch_W(u[i], u[n + i]) * hx * hy;
      for (int c = 0; c < 2; c++) {
        const double *uc = u + c * n;
        if (per || ix < nx - 1) {
          double gx = (uc[(size_t)iy * nx + (ix + 1) % nx] - uc[i]) / hx;
          e += 0.5 * eps * eps * gx * gx * wy * hx * hy;
        }
        if (ny > 1 && (per || iy < ny - 1)) {
          double gy = (uc[(size_t)((iy + 1) % ny) * nx + ix] - uc[i]) / hy;
          e += 0.5 * eps * eps * gy * gy * wx * hx * hy;
        }
      }
    }
  }
  return e;
}

/* One time step of the vector model: for each component the iteration of
 * oracle_step (same operators, same readings), coupled through g. */
int oracle_vch_step(const or_grid *g, const or_params *p, double *u, const double *u_prev, or_info *info) {
  if (!grid_ok(g) || !p || !u) return -1;
  if (!(p->eps > 0) || !(p->dt > 0) || !(p->sigma0 > 0)) return -1;
  const size_t n = (size_t)g->nx * g->ny;
  const int bdf2 = (p->stepper == OR_BDF2) && u_prev != NULL;
  /* variable-step BDF2 as in oracle_step */
  const double w = (p->omega > 0.0) ? p->omega : 1.0;
  const double rc0 = (1.0 + w) * (1.0 + w) / (1.0 + 2.0 * w), rc1 = -w * w / (1.0 + 2.0 * w);
  const double a = (bdf2 ? (1.0 + w) / (1.0 + 2.0 * w) : 1.0) * p->dt;
  double s1, s2, sigma;
  stepper_params(p->eps, a, p->sigma0, &s1, &s2, &sigma);
  const double al1 = 1.0 / sqrt(s1), al2 = 1.0 / sqrt(s2);
  const double kappa = a / s1;
  const size_t n2 = 2 * n;
  double *vn = (double *)malloc(sizeof(double) * n2);
  double *R = (double *)malloc(sizeof(double) * n2);
  double *v = (double *)malloc(sizeof(double) * n2);
  double *gk = (double *)malloc(sizeof(double) * n2);
  double *vnew = (double *)malloc(sizeof(double) * n2);
  double *rhs = (double *)malloc(sizeof(double) * n);
  double *c1 = (double *)malloc(sizeof(double) * n);
  double *t1 = (double *)malloc(sizeof(double) * n);
  double *t2 = (double *)malloc(sizeof(double) * n);
  double *dv = (double *)malloc(sizeof(double) * n);
  double *q = (double *)malloc(sizeof(double) * n);
  if (!vn || !R || !v || !gk || !vnew || !rhs || !c1 || !t1 || !t2 || !dv || !q) return -2;

  for (int c = 0; c < 2; c++)
    for (size_t i = 0; i < n; i++) vn[c * n + i] = u[c * n + i] - OR_Z[2][c];
  for (int c = 0; c < 2; c++) {
    for (size_t i = 0; i < n; i++) {
      const double vp = bdf2 ? u_prev[c * n + i] - OR_Z[2][c] : 0.0;
      rhs[i] = !bdf2 ? vn[c * n + i] : (w == 1.0 ? (4.0 * vn[c * n + i] - vp) / 3.0 : rc0 * vn[c * n + i] + rc1 * vp);
    }
    Ainv(g, al2, rhs, t2, t1);
    Ainv(g, al1, t2, R + c * n, t1);
  }
  memcpy(v, p->init == OR_INIT_LINEAR ? R : vn, sizeof(double) * n2);

  int k = 0;
  double res = 0.0;
  for (;;) {
    for (size_t i = 0; i < n; i++) {
      double gw[2];
      oracle_vch_gradW(v[i] + OR_Z[2][0], v[n + i] + OR_Z[2][1], gw);
      gk[i] = gw[0] - sigma * v[i];
      gk[n + i] = gw[1] - sigma * v[n + i];
    }
    res = 0.0;
    for (int c = 0; c < 2; c++) {
      const double *gc = gk + c * n, *vc = v + c * n, *Rc = R + c * n;
      Ainv(g, al1, gc, c1, t1);
      Dop(g, al1, gc, t2, t1, n);
      for (size_t i = 0; i < n; i++) c1[i] = c1[i] - gc[i] + t2[i];
      Ainv(g, al2, c1, t2, t1);
      Dop(g, al1, vc, dv, t1, n);
      for (size_t i = 0; i < n; i++) q[i] = vc[i] - dv[i];
      Dop(g, al2, q, c1, t1, n);
      for (size_t i = 0; i < n; i++) {
        const double x = Rc[i] + kappa * t2[i] + dv[i] + c1[i];
        const double e = fabs(x - vc[i]);
        if (e > res) res = e;
        vnew[c * n + i] = x;
      }
    }
    memcpy(v, vnew, sizeof(double) * n2);
    k++;
    if (p->fixed_iters > 0) {
      if (k >= p->fixed_iters) break;
    } else if (res < p->tol || k >= p->max_iter) {
      break;
    }
  }
  for (int c = 0; c < 2; c++)
    for (size_t i = 0; i < n; i++) u[c * n + i] = v[c * n + i] + OR_Z[2][c];
  if (info) {
    info->iters = k;
    info->residual = res;
    info->mass = oracle_mass(g, u);
    info->mass2 = oracle_mass(g, u + n);
    info->energy = oracle_vch_energy(g, p->eps, u);
    info->s1 = s1;
    info->s2 = s2;
    info->sigma = sigma;
  }
  free(vn); free(R); free(v); free(gk); free(vnew); free(rhs);
  free(c1); free(t1); free(t2); free(dv); free(q);
  return (p->fixed_iters <= 0 && res >= p->tol) ? 1 : 0;
}

/* nsteps steps of the vector model (BDF2: BE first step, as oracle_solve). */
int oracle_vch_solve(const or_grid *g, const or_params *p, double *u, int nsteps, or_info *infos) {
  if (!grid_ok(g) || !p || !u || nsteps < 0) return -1;
  const size_t n2 = 2 * (size_t)g->nx * g->ny;
  double *prev = (double *)malloc(sizeof(double) * n2);
  double *cur = (double *)malloc(sizeof(double) * n2);
  int status = 0;
  for (int s = 0; s < nsteps; s++) {
    memcpy(cur, u, sizeof(double) * n2);
    int rc = oracle_vch_step(g, p, u, s == 0 ? NULL : prev, infos ? &infos[s] : NULL);
    if (rc < 0) { status = rc; break; }
    if (rc > 0) status = 1;
    memcpy(prev, cur, sizeof(double) * n2);
  }
  free(prev);
  free(cur);
  return status;
}
