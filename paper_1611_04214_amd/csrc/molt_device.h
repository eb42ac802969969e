// molt_device.h -- device code shared by the HIP translation units of libmolt:
// the pass programs, the per-thread line segment, the boundary solve and the
// bodies of the line-pass kernels (block index passed explicitly, so that the
// single-problem kernels and the batched kernels run the same code).
//
// The MOL^T Cahn-Hilliard hot path: the line inverse L^{-1} =
// (I - d^2/alpha^2)^{-1} of Sec. 3.2 along x-lines and y-lines, fused with the
// pointwise work of the fixed-point iteration of Sec. 5.1.
//
// One line inverse, for nodes j = 0..n-1 with J^L_j, J^R_j the order-M local
// quadratures (centred stencils; J^L_0 = 0, and J^R_{n-1} = 0 when the line is
// not periodic):
//   S^L_j = d S^L_{j-1} + J^L_j,   S^R_j = d S^R_{j+1} + J^R_j        (eqs. IL, IR)
//   w_j   = (S^L_j + S^R_j)/2 + B_a d^j + B_b d^{N-j}                 (eq. L_Inverse)
// with B_a, B_b from the boundary 2x2 solve (FP64).  The recurrences are
// evaluated as a parallel scan: each thread owns K consecutive nodes, first
// computes its zero-seeded totals, the carries between threads are combined
// (wave shuffles + LDS along x, a per-column FP64 combine kernel along y), and
// a second seeded scan gives the final values.  The boundary terms are folded
// into the seeds: Z^L_j = S^L_j + 2 B_a d^j satisfies the same recurrence, so a
// thread starting at node j0 seeds its scan with d*carry + 2 B_a d^{j0}.
//
// Pass "programs" define the pointwise work around the sweeps: what is swept
// (sin), what is kept per node (ext) and how outputs are formed (fin).
#pragma once
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "molt_internal.h"

// Minimum waves per SIMD requested for the line-pass kernels (caps their VGPRs).
#ifndef MOLT_OCC
#define MOLT_OCC 2
#endif

#define MOLT_PASS_ATTR __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MOLT_OCC)))


namespace molt {

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T dpow(double nu, double e);
template <>
__device__ __forceinline__ float dpow<float>(double nu, double e) {
  return __expf(-(float)(nu * e));
}
template <>
__device__ __forceinline__ double dpow<double>(double nu, double e) {
  return exp(-nu * e);
}

__device__ __forceinline__ int wrapi(int j, int n) {
  int r = j % n;
  return r < 0 ? r + n : r;
}
// j in [-n, 2n): one correction instead of a division
__device__ __forceinline__ int wrap1(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }

// --------------------------------------------------------------------------
// pass programs
//   NR raw input fields a.in[0..NR-1]; need(a, r) says whether field r is read
//   sin(a, r, s):    the F swept fields of a node from its NR raw values
//   ext(a, r, x):    the E values kept on owned nodes for the output
//   fin(a, w, x, o): the NO outputs (a.out[0..NO-1]) from the swept values w;
//                    returns the node's contribution to the residual max.
// The iteration works in u (= v - 1): every linear operator of the scheme
// maps constants to themselves (L^{-1}[1] = 1) or to zero (D, C1), so the
// shift only changes the reaction: g = f(v) - sigma v = u^3 - (1+sigma) u - sigma,
// and the constant drops out of C1 g.
// --------------------------------------------------------------------------
enum ProgId { PROG_SWEEP = 0, PROG_RHS = 1, PROG_P1 = 2, PROG_P2 = 3, PROG_P3 = 4, PROG_P4 = 5, PROG_P1V = 6,
              PROG_P2V = 7, PROG_P2F = 8, PROG_P4F = 9, PROG_RHSW = 10, PROG_P4R = 11 };
// P2F, P4F: P2 and P4 of the full form (first iteration, FP64 restarts) with
// the increment-form inputs left out (fewer registers); RHSW: the rhs read
// from FP32 fields by the FP64 kernels (the setup of an FP32 step, without
// widened copies of u^n and its histories); P4R: P4F writing the re-based FP32
// iterate of an FP32 step; timed under P2, P4, RHS, P4
constexpr int prog_slot(int prog) {
  return prog == PROG_P2F ? PROG_P2
                          : ((prog == PROG_P4F || prog == PROG_P4R) ? PROG_P4 : (prog == PROG_RHSW ? PROG_RHS : prog));
}

template <typename T>
struct ProgSweep {  // w = L^{-1} in0
  static constexpr int F = 1, E = 0, NR = 1, NO = 1;
  static constexpr bool NT = true;
  __device__ static bool need(const PassArgs&, int) { return true; }
  __device__ static void sin(const PassArgs&, const T* r, T* s) { s[0] = r[0]; }
  __device__ static void ext(const PassArgs&, const T*, T*) {}
  __device__ static double fin(const PassArgs&, const T* w, const T*, T* o) {
    o[0] = w[0];
    return 0.0;
  }
};

template <typename T>
struct ProgRhs {  // w = L^{-1} rhs, rhs = u^n (BE), (4u^n - u^{n-1})/3 (BDF2), rc0 u^n + rc1 u^{n-1}
                  // (variable-step BDF2) or (18u^n - 9u^{n-1} + 2u^{n-2})/11 (BDF3)
  static constexpr int F = 1, E = 0, NR = 3, NO = 1;
  static constexpr bool NT = true;
  __device__ static bool need(const PassArgs& a, int r) { return r == 0 || (r == 1 && a.bdf2) || a.bdf2 == 3; }
  __device__ static void sin(const PassArgs& a, const T* r, T* s) {
    if (a.bdf2 == 3)
      s[0] = (T(18) * r[0] - T(9) * r[1] + T(2) * r[2]) * T(1.0 / 11.0);
    else if (a.bdf2 == 2)
      s[0] = (T)a.rc0 * r[0] + (T)a.rc1 * r[1];
    else
      s[0] = a.bdf2 ? (T(4) * r[0] - r[1]) * T(1.0 / 3.0) : r[0];
  }
  __device__ static void ext(const PassArgs&, const T*, T*) {}
  __device__ static double fin(const PassArgs&, const T* w, const T*, T* o) {
    o[0] = w[0];
    return 0.0;
  }
};

template <typename T>
struct ProgRhsW : ProgRhs<T> {};  // ProgRhs on FP32 raw fields (see RawType)

// element type of a program's raw input fields: T, except the FP32 fields the
// FP64 rhs of an FP32 step reads (converted exactly on load)
template <class P, typename T>
struct RawType {
  using type = T;
};
template <>
struct RawType<ProgRhsW<double>, double> {
  using type = float;
};
// element type of a program's outputs: T, except P4R's FP32 fields (each
// output rounded once on store)
template <class P, typename T>
struct OutType {
  using type = T;
};

// reaction part and linear part of the current iterate; the fields hold
// x = u - c (c = a.ushift[0]: 0, or -1 for the shifted variable v = u + 1 of
// eq. CahnHilliard_v), g(x) = f(x + c) - sigma x with f(u) = u^3 - u
//  full form:      e = g(x) (constant dropped when c = 0), lin = x
//  increment form: e = g(p) - g(q) = dl*(p^2 + p q + q^2 - 1 - sigma), lin = dl,
//                  p = base + c + W (current iterate in u), q = p - dl (previous)
// (contraction is spelled out, so every kernel that inlines this rounds alike
// whatever it knows of the arguments)
template <typename T>
__device__ __forceinline__ void react_lin(const PassArgs& a, T base, T W, T dl, T& e, T& lin) {
#pragma clang fp contract(off)
  const T sg = (T)a.sigma;
  const T c = (T)a.ushift[0];
  // both forms, then a select: no branch for the compiler to sink the loads of
  // W and dl into
  const T bu = base + c;
  const T e0 = fma(-sg, base, fma(bu * bu, bu, -bu));
  const T p = base + c + W;
  const T q = p - dl;
  const T e1 = dl * (fma(p, p + q, q * q) - (T(1) + sg));
  const bool full = a.mode == 0;
  e = full ? e0 : e1;
  lin = full ? base : dl;
}

template <typename T>
struct ProgP1 {  // y, alpha1: raw (base, W, dl) -> a1 = Y1 e, b1 = Y1 lin
  static constexpr int F = 2, E = 0, NR = 3, NO = 2;
  static constexpr bool NT = true;
  __device__ static bool need(const PassArgs& a, int r) { return r == 0 || a.mode; }
  __device__ static void sin(const PassArgs& a, const T* r, T* s) { react_lin<T>(a, r[0], r[1], r[2], s[0], s[1]); }
  __device__ static void ext(const PassArgs&, const T*, T*) {}
  __device__ static double fin(const PassArgs&, const T* w, const T*, T* o) {
    o[0] = w[0];
    o[1] = w[1];
    return 0.0;
  }
};

template <typename T>
struct ProgP2 {  // x, alpha1: raw (a1, b1, base, W, dl) -> C = X1(2 a1 - e) - a1, q = b1 + X1(lin - b1)
  static constexpr int F = 2, E = 2, NR = 5, NO = 2;
  static constexpr bool NT = true;
  __device__ static bool need(const PassArgs& a, int r) { return r < 3 || a.mode; }
  __device__ static void sin(const PassArgs& a, const T* r, T* s) {
    T e, lin;
    react_lin<T>(a, r[2], r[3], r[4], e, lin);
    s[0] = T(2) * r[0] - e;
    s[1] = lin - r[1];
  }
  __device__ static void ext(const PassArgs&, const T* r, T* x) {
    x[0] = r[0];
    x[1] = r[1];
  }
  __device__ static double fin(const PassArgs&, const T* w, const T* x, T* o) {
    o[0] = w[0] - x[0];
    o[1] = x[1] + w[1];
    return 0.0;
  }
};

// the reaction of the full form, rounded as react_lin's full branch
template <typename T>
__device__ __forceinline__ T react_full(const PassArgs& a, T base) {
#pragma clang fp contract(off)
  const T sg = (T)a.sigma;
  const T c = (T)a.ushift[0];
  const T bu = base + c;
  return fma(-sg, base, fma(bu * bu, bu, -bu));
}

template <typename T>
struct ProgP2F {  // P2 of the full form: raw (a1, b1, base), e = g(base), lin = base
  static constexpr int F = 2, E = 2, NR = 3, NO = 2;
  static constexpr bool NT = true;
  __device__ static bool need(const PassArgs&, int) { return true; }
  __device__ static void sin(const PassArgs& a, const T* r, T* s) {
    const T e = react_full<T>(a, r[2]);
    s[0] = T(2) * r[0] - e;
    s[1] = r[2] - r[1];
  }
  __device__ static void ext(const PassArgs&, const T* r, T* x) {
    x[0] = r[0];
    x[1] = r[1];
  }
  __device__ static double fin(const PassArgs&, const T* w, const T* x, T* o) {
    o[0] = w[0] - x[0];
    o[1] = x[1] + w[1];
    return 0.0;
  }
};

template <typename T>
struct ProgP3 {  // y, alpha2: raw (C, q) -> m = Y2(q + kappa C) - q, n = Y2 q
  static constexpr int F = 2, E = 1, NR = 2, NO = 2;
  // cacheable outputs, read back by P4 (4096^2: P3 56 -> 50 us, P4 84 -> 83 us)
  static constexpr bool NT = false;
  __device__ static bool need(const PassArgs&, int) { return true; }
  __device__ static void sin(const PassArgs& a, const T* r, T* s) {
    s[0] = r[1] + (T)a.kappa * r[0];
    s[1] = r[1];
  }
  __device__ static void ext(const PassArgs&, const T* r, T* x) { x[0] = r[1]; }
  __device__ static double fin(const PassArgs&, const T* w, const T* x, T* o) {
    o[0] = w[0] - x[0];
    o[1] = w[1];
    return 0.0;
  }
};

template <typename T>
struct ProgP4 {  // x, alpha2: raw (m, n, dl|R, W) -> dl' = (dl|R) + X2 m - n ; W' = W + dl' (| dl')
  static constexpr int F = 1, E = 3, NR = 4, NO = 2;
  static constexpr bool NT = false;  // (see the note at st16_nt)
  __device__ static bool need(const PassArgs& a, int r) { return r < 3 || a.mode; }
  __device__ static void sin(const PassArgs&, const T* r, T* s) { s[0] = r[0]; }
  __device__ static void ext(const PassArgs& a, const T* r, T* x) {
    x[0] = r[1];
    x[1] = r[2];
    x[2] = a.mode ? r[3] : T(0);
  }
  __device__ static double fin(const PassArgs&, const T* w, const T* x, T* o) {
    const T dn = x[1] + w[0] - x[0];
    o[0] = dn;
    o[1] = x[2] + dn;
    return fabs((double)dn);
  }
};

template <typename T>
struct ProgP4F {  // P4 of the full form: raw (m, n, R) -> dl' = R + X2 m - n, W' = dl'
  static constexpr int F = 1, E = 2, NR = 3, NO = 2;
  static constexpr bool NT = false;
  __device__ static bool need(const PassArgs&, int) { return true; }
  __device__ static void sin(const PassArgs&, const T* r, T* s) { s[0] = r[0]; }
  __device__ static void ext(const PassArgs&, const T* r, T* x) {
    x[0] = r[1];
    x[1] = r[2];
  }
  __device__ static double fin(const PassArgs&, const T* w, const T* x, T* o) {
    const T dn = x[1] + w[0] - x[0];
    o[0] = dn;
    o[1] = T(0) + dn;  // (P4's W' = 0 + dl': the same zero signs)
    return fabs((double)dn);
  }
};

template <typename T>
struct ProgP4R {  // P4F of an FP64 iteration in an FP32 step: raw (m, n, R), the iterate's base read
                  // late (see Late) -> the FP32 fields the FP32 iterations continue from (see
                  // OutType): dl' = R + X2 m - n, v = base + (0 + dl') split into fl32(v) and the rest
  static constexpr int F = 1, E = 2, NR = 3, NO = 3;
  static constexpr bool NT = false;
  __device__ static bool need(const PassArgs&, int) { return true; }
  __device__ static void sin(const PassArgs&, const T* r, T* s) { s[0] = r[0]; }
  __device__ static void ext(const PassArgs&, const T* r, T* x) {
    x[0] = r[1];
    x[1] = r[2];
  }
  // x[2]: the late input, the base of the iterate
  __device__ static double fin(const PassArgs&, const T* w, const T* x, T* o) {
    const T dn = x[1] + w[0] - x[0];
    const T wn = T(0) + dn;  // (P4F's W', which the FP64 iterate holds)
    const T v = x[2] + wn;
    const T b = (T)(float)v;
    o[0] = wn;     // dl', rounded to FP32 by the store (dl' = W' in the full form)
    o[1] = v - b;  // the FP32 running sum starts at the rounding error of the base
    o[2] = b;      // the FP32 base
    return fabs((double)dn);
  }
};

// inputs a program reads only where it forms its outputs (a.in[NR], ...),
// appended to its kept values: no registers held across the pass
template <class P>
struct Late {
  static constexpr int n = 0;
};
template <typename T>
struct Late<ProgP4R<T>> {
  static constexpr int n = 1;
};

// Vector model: the reaction and linear parts (e, lin) of both components are
// formed by a pointwise pre-pass (vch_react_body); P1 and P2 then sweep them
// like any stacked pair of fields.
template <typename T>
struct ProgP1V {  // y, alpha1: raw (e, lin) -> a1 = Y1 e, b1 = Y1 lin
  static constexpr int F = 2, E = 0, NR = 2, NO = 2;
  static constexpr bool NT = true;
  __device__ static bool need(const PassArgs&, int) { return true; }
  __device__ static void sin(const PassArgs&, const T* r, T* s) {
    s[0] = r[0];
    s[1] = r[1];
  }
  __device__ static void ext(const PassArgs&, const T*, T*) {}
  __device__ static double fin(const PassArgs&, const T* w, const T*, T* o) {
    o[0] = w[0];
    o[1] = w[1];
    return 0.0;
  }
};

template <typename T>
struct ProgP2V {  // x, alpha1: raw (a1, b1, e, lin) -> C = X1(2 a1 - e) - a1, q = b1 + X1(lin - b1)
  static constexpr int F = 2, E = 2, NR = 4, NO = 2;
  static constexpr bool NT = true;
  __device__ static bool need(const PassArgs&, int) { return true; }
  __device__ static void sin(const PassArgs&, const T* r, T* s) {
    s[0] = T(2) * r[0] - r[2];
    s[1] = r[3] - r[1];
  }
  __device__ static void ext(const PassArgs&, const T* r, T* x) {
    x[0] = r[0];
    x[1] = r[1];
  }
  __device__ static double fin(const PassArgs&, const T* w, const T* x, T* o) {
    o[0] = w[0] - x[0];
    o[1] = x[1] + w[1];
    return 0.0;
  }
};

template <int P, typename T>
struct ProgOf;
template <typename T> struct ProgOf<PROG_P1V, T> { using type = ProgP1V<T>; };
template <typename T> struct ProgOf<PROG_P2V, T> { using type = ProgP2V<T>; };
template <typename T> struct ProgOf<PROG_SWEEP, T> { using type = ProgSweep<T>; };
template <typename T> struct ProgOf<PROG_RHS, T> { using type = ProgRhs<T>; };
template <typename T> struct ProgOf<PROG_P1, T> { using type = ProgP1<T>; };
template <typename T> struct ProgOf<PROG_P2, T> { using type = ProgP2<T>; };
template <typename T> struct ProgOf<PROG_P3, T> { using type = ProgP3<T>; };
template <typename T> struct ProgOf<PROG_P4, T> { using type = ProgP4<T>; };
template <typename T> struct ProgOf<PROG_P2F, T> { using type = ProgP2F<T>; };
template <typename T> struct ProgOf<PROG_P4F, T> { using type = ProgP4F<T>; };
template <typename T> struct ProgOf<PROG_RHSW, T> { using type = ProgRhsW<T>; };
template <typename T> struct ProgOf<PROG_P4R, T> { using type = ProgP4R<T>; };
template <>
struct OutType<ProgP4R<double>, double> {
  using type = float;
};

// field f of a program's raw inputs, or field 0 (always read, same size) in
// place of a field it does not read: loads are then unconditional, so the
// compiler can issue all of a thread's loads before the first use, and the
// stand-in loads hit the cache lines of field 0's
template <typename T, class P>
__device__ __forceinline__ const typename RawType<P, T>::type* raw_ptr(const PassArgs& a, int f) {
  return (const typename RawType<P, T>::type*)(P::need(a, f) ? a.in[f] : a.in[0]);
}

// raw values of one node (scalar loads; fields the program does not read are 0)
template <typename T, class P>
__device__ __forceinline__ void load_raw(const PassArgs& a, size_t i, T* r) {
#pragma unroll
  for (int f = 0; f < P::NR; ++f) {
    const T v = (T)raw_ptr<T, P>(a, f)[i];
    r[f] = P::need(a, f) ? v : T(0);
  }
}

// 16-byte vector access of 16/sizeof(T) consecutive elements
// (FP32: a streaming load; the x-pass reads each input once, and at 4096^2 the
// hint took the P2 x-pass from 85.6 to 83.3 us)
__device__ __forceinline__ void ld16(const float* p, float* o) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 v = __builtin_nontemporal_load((const v4*)p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld16(const double* p, double* o) {
  const double2 v = *(const double2*)p;
  o[0] = v.x; o[1] = v.y;
}
__device__ __forceinline__ void st16(float* p, const float* o) { *(float4*)p = make_float4(o[0], o[1], o[2], o[3]); }
__device__ __forceinline__ void st16(double* p, const double* o) { *(double2*)p = make_double2(o[0], o[1]); }

// Nontemporal (streaming) stores for the line passes' outputs: on the MI355X
// they cut the x-pass P2 from 98 to 84 us and the P1 y-pass final kernel from
// 71 to 60 us at 4096^2.  A program sets NT = false when the pass that reads
// its outputs next does better with them cached (P4's outputs: the P1 y-pass
// totals kernel ran 41 -> 46 us after streamed stores).
typedef float molt_f4v __attribute__((ext_vector_type(4)));
typedef double molt_d2v __attribute__((ext_vector_type(2)));
// 16/sizeof(T) consecutive raw values of field f at element `off` (the FP32
// fields of an FP64 program: one 8-byte load of two floats, widened)
template <typename T, class P>
__device__ __forceinline__ void ld16_raw(const PassArgs& a, int f, size_t off, T* o) {
  using R = typename RawType<P, T>::type;
  const R* p = raw_ptr<T, P>(a, f) + off;
  if constexpr (std::is_same<R, T>::value) {
    ld16(p, o);
  } else {
    static_assert(sizeof(T) == 8 && sizeof(R) == 4, "FP32 inputs of FP64 programs only");
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 x = *(const v2*)p;
    o[0] = (T)x.x;
    o[1] = (T)x.y;
  }
}

__device__ __forceinline__ void st16_nt(float* p, const float* o) {
  const molt_f4v v = {o[0], o[1], o[2], o[3]};
  __builtin_nontemporal_store(v, (molt_f4v*)p);
}
__device__ __forceinline__ void st16_nt(double* p, const double* o) {
  const molt_d2v v = {o[0], o[1]};
  __builtin_nontemporal_store(v, (molt_d2v*)p);
}
template <bool NT, typename T>
__device__ __forceinline__ void st16_out(T* p, const T* o) {
  if constexpr (NT) st16_nt(p, o); else st16(p, o);
}
template <bool NT, typename T>
__device__ __forceinline__ void st1_out(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
}
// output f of a program: 16/sizeof(T) values at element `off`, or one value at
// element `i` (FP32 outputs of an FP64 program: rounded, one 8-byte store)
template <typename T, class P>
__device__ __forceinline__ void st16_prog(const PassArgs& a, int f, size_t off, const T* o) {
  using O = typename OutType<P, T>::type;
  if constexpr (std::is_same<O, T>::value) {
    st16_out<P::NT>((T*)a.out[f] + off, o);
  } else {
    static_assert(sizeof(T) == 8 && sizeof(O) == 4, "FP32 outputs of FP64 programs only");
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 x = {(float)o[0], (float)o[1]};
    *(v2*)((O*)a.out[f] + off) = x;
  }
}
template <typename T, class P>
__device__ __forceinline__ void st1_prog(const PassArgs& a, int f, size_t i, T v) {
  using O = typename OutType<P, T>::type;
  st1_out<P::NT>((O*)a.out[f] + i, (O)v);
}

// Corrections an x-pass applies to the raw fields it reads from a deferred
// y-pass (see YCorr): for its row, the factors 1/2 d^(j - j0s) and
// 1/2 d^(jls - j) and the seed rows of the row's segment.
template <typename T>
struct RowCorr {
  // seed rows of fields 0 and 1 (named members, not arrays: a field index the
  // compiler cannot resolve then selects a register instead of indexing the
  // object in scratch memory)
  const T* sL0;
  const T* sL1;
  const T* sR0;
  const T* sR1;
  T cL, cR;
  int nf;  // 0: nothing to correct
  __device__ __forceinline__ const T* seedL(int f) const { return f == 0 ? sL0 : sL1; }
  __device__ __forceinline__ const T* seedR(int f) const { return f == 0 ? sR0 : sR1; }
  __device__ void init(const YCorr& yc, int line) {
    nf = yc.seeds != nullptr ? yc.nf : 0;
    sL0 = sL1 = sR0 = sR1 = nullptr;
    cL = cR = T(0);
    if (nf == 0) return;
    const int b = line / yc.ny, j = line - b * yc.ny;
    const int seg = j / yc.S;
    const int j0s = seg * yc.S;
    const int jls = min(j0s + yc.S - 1, yc.ny - 1);
    cL = T(0.5) * dpow<T>(yc.nu, (double)(j - j0s));
    cR = T(0.5) * dpow<T>(yc.nu, (double)(jls - j));
    const size_t plane = (size_t)yc.nseg * yc.nx;
    const T* base0 = (const T*)yc.seeds + ((size_t)(b * yc.nf) * 2) * plane + (size_t)seg * yc.nx;
    const T* base1 = (const T*)yc.seeds + ((size_t)(b * yc.nf + (yc.nf > 1 ? 1 : 0)) * 2) * plane + (size_t)seg * yc.nx;
    sL0 = base0;
    sR0 = base0 + plane;
    sL1 = base1;
    sR1 = base1 + plane;
  }
  // raw values r of column col (fields f < nf corrected)
  template <int NR>
  __device__ __forceinline__ void apply(int col, T* r) const {
#pragma unroll
    for (int f = 0; f < (NR < 2 ? NR : 2); ++f)
      if (f < nf) r[f] += cL * seedL(f)[col] + cR * seedR(f)[col];
  }
};

// --------------------------------------------------------------------------
// Per-thread line segment: sweep inputs on nodes j0-H .. j0+K+H-1, the two
// local quadratures on the K owned nodes, zero-seeded totals and the final
// seeded scans.  `stride` is the element distance between consecutive nodes
// of the line (1 along x, nx along y); `lbase` the element index of node 0.
// With `vec` (stride 1, 16-byte aligned fields, line length a multiple of
// 16/sizeof(T)) owned nodes are read with 16-byte loads.
// --------------------------------------------------------------------------
template <typename T, class P, int K, int M, bool PER>
struct Seg {
  static constexpr int H = M / 2, F = P::F, E = P::E, NR = P::NR, W = K + 2 * H;
  static constexpr int V = 16 / (int)sizeof(T);
  T JL[F][K], JR[F][K];
  T jln[F];                    // periodic: J^L of the cell ending at node n (= node 0)
  T ex[E > 0 ? E : 1][K];      // kept values of the owned nodes

  __device__ void build(const LineCoef& c, const PassArgs& a, size_t lbase, size_t stride, int j0, bool vec) {
    T s[F][W];
    window(c, a, lbase, stride, j0, vec, s);
    RowCorr<T> none;
    none.nf = 0;
    stencils(c, a, lbase, stride, j0, s, none);
  }

  // swept values on nodes j0-H .. j0+K+H-1 (and the kept values of the owned nodes)
  __device__ void window(const LineCoef& c, const PassArgs& a, size_t lbase, size_t stride, int j0, bool vec,
                         T (&s)[F][W]) {
    const int n = c.n;
    constexpr bool per = PER;
    const bool near = n >= K + H;  // then every window index is within one period
    if (vec && j0 + K <= n) {
#pragma unroll
      for (int q = 0; q < K / V; ++q) {
        T r[NR][V];
#pragma unroll
        for (int f = 0; f < NR; ++f) ld16_raw<T, P>(a, f, lbase + (size_t)(j0 + q * V), r[f]);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          T rv[NR], sv[F], xv[E > 0 ? E : 1];
#pragma unroll
          for (int f = 0; f < NR; ++f) rv[f] = P::need(a, f) ? r[f][v] : T(0);
          P::sin(a, rv, sv);
#pragma unroll
          for (int f = 0; f < F; ++f) s[f][H + q * V + v] = sv[f];
          if constexpr (E > 0) {
            P::ext(a, rv, xv);
#pragma unroll
            for (int e = 0; e < E; ++e) ex[e][q * V + v] = xv[e];
          }
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = j0 + k;
        const int jj = per ? (near ? wrap1(j, n) : wrapi(j, n)) : min(j, n - 1);
        T rv[NR], sv[F], xv[E > 0 ? E : 1];
        load_raw<T, P>(a, lbase + (size_t)jj * stride, rv);
        P::sin(a, rv, sv);
#pragma unroll
        for (int f = 0; f < F; ++f) s[f][H + k] = sv[f];
        if constexpr (E > 0) {
          P::ext(a, rv, xv);
#pragma unroll
          for (int e = 0; e < E; ++e) ex[e][k] = xv[e];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) {  // halo nodes (ends of non-periodic lines: clamped, replaced below)
      const int kk = k < H ? k : K + k;
      const int j = j0 - H + kk;
      const int jj = per ? (near ? wrap1(j, n) : wrapi(j, n)) : min(max(j, 0), n - 1);
      T rv[NR], sv[F];
      load_raw<T, P>(a, lbase + (size_t)jj * stride, rv);
      P::sin(a, rv, sv);
#pragma unroll
      for (int f = 0; f < F; ++f) s[f][kk] = sv[f];
    }
  }

  // J^L, J^R on the owned nodes from the window values s (nodes j0-H ..
  // j0+K+H-1); boundary nodes of non-periodic lines are redone in FP64
  __device__ __attribute__((always_inline)) void stencils(const LineCoef& c, const PassArgs& a, size_t lbase, size_t stride, int j0,
                           const T (&s)[F][W], const RowCorr<T>& rc) {
    const int n = c.n;
    constexpr bool per = PER;
    T wl[M + 1], wr[M + 1];
#pragma unroll
    for (int i = 0; i <= M; ++i) {
      wl[i] = (T)c.wl[i];
      wr[i] = (T)c.wr[i];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = j0 + k;
      const bool real = j < n;
#pragma unroll
      for (int f = 0; f < F; ++f) {
        T l = T(0), r = T(0);
#pragma unroll
        for (int i = 0; i <= M; ++i) {
          l += wl[i] * s[f][k + i];
          r += wr[i] * s[f][k + i];
        }
        if (k == 0) jln[f] = l;
        JL[f][k] = (real && j != 0) ? l : T(0);
        JR[f][k] = (real && (per || j != n - 1)) ? r : T(0);
      }
    }
    if constexpr (!PER) {
      if (j0 < H || j0 + K + H > n) boundary_nodes(c, a, lbase, stride, j0, rc);
    }
  }

  // Nodes whose centred window leaves a non-periodic line (j < H or j > n-1-H).
  // The window is completed by ghost values extrapolated with the degree-M
  // polynomial through the M+1 end nodes; the extrapolation weights are large
  // (up to ~2800 for M=6), so the ghosts and these few stencils are formed in
  // FP64 and only the result is rounded to T.  The in-range window values are
  // reloaded here (only the threads at the two ends of a line get here), so
  // the window array of the interior path is not kept alive.
  // (rc: the x-pass's row corrections, applied to every reloaded value; nf = 0 for none)
  __device__ __attribute__((always_inline)) void boundary_nodes(const LineCoef& c, const PassArgs& a, size_t lbase, size_t stride, int j0,
                                 const RowCorr<T>& rc) {
    const int n = c.n;
    double gl[F][H], gr[F][H];
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int g = 0; g < H; ++g) gl[f][g] = gr[f][g] = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side == 0 ? (j0 >= H) : (j0 + K + H <= n)) continue;
      double e[F][M + 1];
#pragma unroll
      for (int i = 0; i <= M; ++i) {
        T rv[NR], sv[F];
        const int jn = side == 0 ? i : n - 1 - M + i;
        load_raw<T, P>(a, lbase + (size_t)jn * stride, rv);
        rc.template apply<NR>(jn, rv);
        P::sin(a, rv, sv);
#pragma unroll
        for (int f = 0; f < F; ++f) e[f][i] = (double)sv[f];
      }
#pragma unroll
      for (int f = 0; f < F; ++f)
#pragma unroll
        for (int g = 0; g < H; ++g) {
          double acc = 0.0;
#pragma unroll
          for (int i = 0; i <= M; ++i) acc += (side == 0 ? c.ghostL[g][i] : c.ghostR[g][i]) * e[f][i];
          if (side == 0)
            gl[f][g] = acc;
          else
            gr[f][g] = acc;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = j0 + k;
      if (j < n && (j < H || j > n - 1 - H)) {
#pragma unroll
        for (int f = 0; f < F; ++f) {
          double l = 0.0, r = 0.0;
#pragma unroll
          for (int i = 0; i <= M; ++i) {
            const int jw = j - H + i;
            T rv[NR], sv[F];
            const int jc = min(max(jw, 0), n - 1);
            load_raw<T, P>(a, lbase + (size_t)jc * stride, rv);
            rc.template apply<NR>(jc, rv);
            P::sin(a, rv, sv);
            double v = (double)sv[f];
#pragma unroll
            for (int g = 1; g <= H; ++g) {
              v = (jw == -g) ? gl[f][g - 1] : v;
              v = (jw == n - 1 + g) ? gr[f][g - 1] : v;
            }
            l += c.wl[i] * v;
            r += c.wr[i] * v;
          }
          JL[f][k] = (j != 0) ? (T)l : T(0);
          JR[f][k] = (j != n - 1) ? (T)r : T(0);
        }
      }
    }
  }

  // zero-seeded totals: AL at the thread's last real node, AR at its first node
  __device__ void totals(T d, int j0, int n, T* AL, T* AR) const {
    const int jlast = min(j0 + K - 1, n - 1);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      T x = T(0), xl = T(0);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        x = d * x + JL[f][k];
        if (j0 + k == jlast) xl = x;
      }
      AL[f] = xl;
      T y = T(0);
#pragma unroll
      for (int k = K - 1; k >= 0; --k) y = d * y + JR[f][k];
      AR[f] = y;
    }
  }

  // seeded scans; w[f][k] = (Z^L + Z^R)/2
  __device__ void finalize(T d, int j0, int n, const T* gL, const T* gR, T (&w)[F][K]) const {
    const int jlast = min(j0 + K - 1, n - 1);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      T x = T(0);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        x = (k == 0) ? (JL[f][0] + gL[f]) : (d * x + JL[f][k]);
        w[f][k] = x;
      }
      T y = T(0);
#pragma unroll
      for (int k = K - 1; k >= 0; --k) {
        const int j = j0 + k;
        y = (j > jlast) ? T(0) : ((j == jlast) ? (JR[f][k] + gR[f]) : (d * y + JR[f][k]));
        w[f][k] = T(0.5) * (w[f][k] + y);
      }
    }
  }

  // outputs of the owned nodes; returns the residual max over them
  __device__ double store(const PassArgs& a, size_t lbase, size_t stride, int j0, int n, bool vec,
                          const T (&w)[F][K]) const {
    constexpr int NO = P::NO;
    double res = 0.0;
    if (vec && j0 + K <= n) {
#pragma unroll
      for (int q = 0; q < K / V; ++q) {
        T o[NO][V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int k = q * V + v;
          T wk[F], xk[E > 0 ? E : 1], ok[NO];
#pragma unroll
          for (int f = 0; f < F; ++f) wk[f] = w[f][k];
#pragma unroll
          for (int e = 0; e < E; ++e) xk[e] = ex[e][k];
          res = fmax(res, P::fin(a, wk, xk, ok));
#pragma unroll
          for (int f = 0; f < NO; ++f) o[f][v] = ok[f];
        }
#pragma unroll
        for (int f = 0; f < NO; ++f) st16_prog<T, P>(a, f, lbase + (size_t)(j0 + q * V), o[f]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = j0 + k;
        if (j < n) {
          T wk[F], xk[E > 0 ? E : 1], ok[NO];
#pragma unroll
          for (int f = 0; f < F; ++f) wk[f] = w[f][k];
#pragma unroll
          for (int e = 0; e < E; ++e) xk[e] = ex[e][k];
          res = fmax(res, P::fin(a, wk, xk, ok));
#pragma unroll
          for (int f = 0; f < NO; ++f) st1_prog<T, P>(a, f, lbase + (size_t)j * stride, ok[f]);
        }
      }
    }
    return res;
  }
};

// Boundary coefficients of one line from its zero-seeded totals (Sec. 3.2).
//  TLl = S^L_{n-1}, TRl = S^R_0 (zero-seeded), jlnv = J^L of the cell ending at
//  node N (periodic only).  I_N = IL~_N / 2, I_0 = IR~_0 / 2.
__device__ __forceinline__ void boundary_terms(const LineCoef& c, double TLl, double TRl, double jlnv,
                                               double& Ba, double& Bb) {
  const double d = c.d, mu = c.mu;
  if (c.bc == MOLT_BC_PERIODIC) {
    const double IN = 0.5 * (d * TLl + jlnv), I0 = 0.5 * TRl;
    Ba = IN / (1.0 - mu);
    Bb = I0 / (1.0 - mu);
  } else {
    const double IN = 0.5 * TLl, I0 = 0.5 * TRl;
    const double den = 1.0 - mu * mu;
    if (c.bc == MOLT_BC_NEUMANN) {
      Ba = (I0 + mu * IN) / den;
      Bb = (IN + mu * I0) / den;
    } else {
      Ba = (mu * IN - I0) / den;
      Bb = (mu * I0 - IN) / den;
    }
  }
}

// residual: block max written to a per-block slot; a one-block close kernel
// folds the slots (order-independent max) and advances the iteration state.
__device__ inline void residual_block(double r, double* partials, int slot) {
  __shared__ double red[8];  // one per wave, blocks of up to 512 threads
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_down(r, off));
  if (lane == 0) red[wave] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = fmax(b, red[w]);
    partials[slot] = b;
  }
}

// (blocks of up to 1024 threads; the max is order-independent)
__device__ inline void residual_close_body(const double* partials, int nblocks, DevState* st) {
  if (st->done) return;
  __shared__ double red[16];
  double r = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) r = fmax(r, partials[i]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_down(r, off));
  if (lane == 0) red[wave] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double res = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) res = fmax(res, red[w]);
    const int it = st->iters + 1;
    st->iters = it;
    st->last_resid = res;
    if (st->fixed > 0) {
      if (it >= st->fixed) st->done = 1;
    } else if (res < st->tol || it >= st->max_iter) {
      st->done = 1;
    }
  }
}


// The close of an iteration whose P4 x-pass left st->open_parts residual
// partials (nothing when none is pending or the step is done), by the threads
// of one block of any shape; returns the state's done flag after it (block
// uniform, so the caller need not read back the flag it may have just set).
__device__ inline int residual_close_pending(const double* partials, DevState* st) {
  __shared__ int sh_done;
  const int nb = st->open_parts, done0 = st->done;
  if (done0 || nb == 0) return done0;
  __shared__ double red[16];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nt = blockDim.x * blockDim.y * blockDim.z;
  double r = 0.0;
  for (int i = tid; i < nb; i += nt) r = fmax(r, partials[i]);
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_down(r, off));
  if (lane == 0) red[wave] = r;
  __syncthreads();
  if (tid == 0) {
    double res = red[0];
    for (int w = 1; w < (nt >> 6); ++w) res = fmax(res, red[w]);
    const int it = st->iters + 1;
    int done = 0;
    if (st->fixed > 0) {
      if (it >= st->fixed) done = 1;
    } else if (res < st->tol || it >= st->max_iter) {
      done = 1;
    }
    st->iters = it;
    st->last_resid = res;
    st->done = done;
    st->open_parts = 0;
    sh_done = done;
  }
  __syncthreads();
  return sh_done;
}

// --------------------------------------------------------------------------
// x-direction pass: rows are contiguous; TL threads (a multiple of 64) own one
// row, BS/TL rows per block of BS = 256 (or 512, for rows of 512 threads).
// --------------------------------------------------------------------------
// LDS of one x-pass block: F <= 2 swept rows of BS*K nodes, one pad word per 16
template <typename T, int K, int BS = 256>
struct XRow {
  static constexpr int ROW = BS * K;
  static constexpr int PADDED = ROW + ROW / 16;
  static constexpr int ELEMS = 2 * PADDED;
};

template <typename T, int PI, int K, int M, bool PER, int BS = 256>
__device__ __forceinline__ void xpass_body(const LineCoef& c, const PassArgs& a, DevState* st, int nlines, int TL,
                                           double* rpart, int vec, int bx, T* smem) {
  using P = typename ProgOf<PI, T>::type;
  constexpr int F = P::F, E = P::E, NR = P::NR, NO = P::NO, LT = Late<P>::n;
  constexpr int H = M / 2, W = K + 2 * H;
  constexpr int V = 16 / (int)sizeof(T);
  constexpr int ROW = BS * K;  // nodes of all rows of one block
  constexpr int NWB = BS / 64;  // waves per block (and at most as many rows)
  if (st != nullptr && st->done) return;
  __shared__ T sh_tot[F][2][NWB];
  __shared__ double sh_line[NWB][F][3];
  // swept fields (then the swept results) of the block's rows, one padding
  // word per 16 so that a thread's K consecutive nodes sit 17 words from its
  // neighbour's (no bank conflicts)
  T (*sh_row)[ROW + ROW / 16] = reinterpret_cast<T (*)[ROW + ROW / 16]>(smem);  // [F][padded row]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lil = tid / TL;
  const int t = tid - lil * TL;
  const int wl0 = lil * (TL >> 6);
  const int line = bx * (BS / TL) + lil;
  const bool act = line < nlines;
  const int n = c.n;
  const int j0 = t * K;
  const bool has = act && j0 < n;
  const size_t lbase = (size_t)(act ? line : 0) * (size_t)n;
  const int rowoff = lil * TL * K;
  const T d = (T)c.d;
#define MOLT_PAD(e) ((e) + ((e) >> 4))

  Seg<T, P, K, M, PER> seg;
  // corrections of the deferred y-pass whose outputs this pass reads
  RowCorr<T> rc;
  rc.init(a.corr, act ? line : 0);
  constexpr int NC = NR < 2 ? NR : 2;  // raw fields that can be corrected
  // phase A: coalesced loads, the program's pointwise part in the load layout
  if (act) {
    if (vec) {
      // every load of the thread first (positions past the line read its
      // first element and are dropped), then the pointwise part
      T r[K / V][NR][V];
      // the deferred y-pass's seeds are loaded with the raw fields (all
      // loads in flight together) and folded in after the last of them;
      // folding each group as it arrives keeps fewer registers but
      // serializes the loads (FP32 P2 92 -> 117 us at 4096^2).  The FP64 P4
      // folds them as they arrive: that frees the registers for a second
      // block per CU (FP64 P4 at 4096^2: 208 -> 160 us; the FP64 sweeps lose
      // by it, 72 -> 87 us, and P2 does not reach the next occupancy step)
      constexpr bool kEarly = !(sizeof(T) == 8 && prog_slot(PI) == PROG_P4);
      constexpr int KS = kEarly ? K / V : 1;
      T sl[KS][NC][V], sr[KS][NC][V];
#pragma unroll
      for (int it = 0; it < K / V; ++it) {
        const int e0 = (it * TL + t) * V;
        const size_t off = lbase + (size_t)(e0 < n ? e0 : 0);
#pragma unroll
        for (int f = 0; f < NR; ++f) ld16_raw<T, P>(a, f, off, r[it][f]);
        const int ec = e0 < n ? e0 : 0;
        const int is = kEarly ? it : 0;
#pragma unroll
        for (int f = 0; f < NC; ++f)
          if (f < rc.nf) {
            ld16(rc.seedL(f) + ec, sl[is][f]);
            ld16(rc.seedR(f) + ec, sr[is][f]);
            if constexpr (!kEarly) {
#pragma unroll
              for (int v = 0; v < V; ++v) r[it][f][v] += rc.cL * sl[0][f][v] + rc.cR * sr[0][f][v];
            }
          }
      }
      if (kEarly && rc.nf > 0) {
#pragma unroll
        for (int it = 0; it < K / V; ++it)
#pragma unroll
          for (int f = 0; f < NC; ++f)
            if (f < rc.nf) {
#pragma unroll
              for (int v = 0; v < V; ++v) r[it][f][v] += rc.cL * sl[it][f][v] + rc.cR * sr[it][f][v];
            }
      }
#pragma unroll
      for (int it = 0; it < K / V; ++it) {
        const int e0 = (it * TL + t) * V;
        if (e0 < n) {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            T rv[NR], sv[F], xv[E > 0 ? E : 1];
#pragma unroll
            for (int f = 0; f < NR; ++f) rv[f] = P::need(a, f) ? r[it][f][v] : T(0);
            P::sin(a, rv, sv);
#pragma unroll
            for (int f = 0; f < F; ++f) sh_row[f][MOLT_PAD(rowoff + e0 + v)] = sv[f];
            if constexpr (E > 0) {
              P::ext(a, rv, xv);
#pragma unroll
              for (int e = 0; e < E; ++e) seg.ex[e][it * V + v] = xv[e];
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int it = 0; it < K; ++it) {
        const int e = it * TL + t;
        if (e < n) {
          T rv[NR], sv[F], xv[E > 0 ? E : 1];
          load_raw<T, P>(a, lbase + (size_t)e, rv);
          rc.template apply<NR>(e, rv);
          P::sin(a, rv, sv);
#pragma unroll
          for (int f = 0; f < F; ++f) sh_row[f][MOLT_PAD(rowoff + e)] = sv[f];
          if constexpr (E > 0) {
            P::ext(a, rv, xv);
#pragma unroll
            for (int q = 0; q < E; ++q) seg.ex[q][it] = xv[q];
          }
        }
      }
    }
  }
  __syncthreads();

  // phase B: each thread's window of K + 2H nodes from LDS, local quadratures
  T AL[F], AR[F];
  if (has) {
    T sw[F][W];
    const bool near = n >= K + H;  // then one wrap suffices
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int j = j0 - H + k;
      int jj;
      if (PER)
        jj = near ? (j < 0 ? j + n : (j >= n ? j - n : j)) : wrapi(j, n);
      else
        jj = min(max(j, 0), n - 1);
#pragma unroll
      for (int f = 0; f < F; ++f) sw[f][k] = sh_row[f][MOLT_PAD(rowoff + jj)];
    }
    seg.stencils(c, a, lbase, 1, j0, sw, rc);
    seg.totals(d, j0, n, AL, AR);
  } else {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      AL[f] = T(0);
      AR[f] = T(0);
      seg.jln[f] = T(0);
    }
  }

  // carries between threads of the line: multiplier m = d^K per thread
  const T m = dpow<T>(c.nu, (double)K);
  T mp[6];
  mp[0] = m;
#pragma unroll
  for (int s = 1; s < 6; ++s) mp[s] = mp[s - 1] * mp[s - 1];
  const T m64 = mp[5] * mp[5];
  T exL[F], exR[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    T xL = AL[f], xR = AR[f];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int off = 1 << s;
      T yL = __shfl_up(xL, off);
      T yR = __shfl_down(xR, off);
      if (lane >= off) xL += mp[s] * yL;
      if (lane + off < 64) xR += mp[s] * yR;
    }
    T eL = __shfl_up(xL, 1);
    T eR = __shfl_down(xR, 1);
    exL[f] = lane == 0 ? T(0) : eL;
    exR[f] = lane == 63 ? T(0) : eR;
    if (lane == 63) sh_tot[f][0][wave] = xL;
    if (lane == 0) sh_tot[f][1][wave] = xR;
  }
  __syncthreads();
  const int nw = TL >> 6, wv = t >> 6;
  const T mlane = dpow<T>(c.nu, (double)K * lane);
  const T mlane_r = dpow<T>(c.nu, (double)K * (63 - lane));
  T cL[F], cR[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    T CL = T(0), CR = T(0);
    for (int w = 0; w < wv; ++w) CL = m64 * CL + sh_tot[f][0][wl0 + w];
    for (int w = nw - 1; w > wv; --w) CR = m64 * CR + sh_tot[f][1][wl0 + w];
    cL[f] = exL[f] + mlane * CL;
    cR[f] = exR[f] + mlane_r * CR;
  }
  // line totals for the boundary solve
  const int tstar = (n - 1) / K;
  if (act && t == tstar) {
    const T dk = dpow<T>(c.nu, (double)(n - 1 - tstar * K + 1));
#pragma unroll
    for (int f = 0; f < F; ++f) sh_line[lil][f][0] = (double)AL[f] + (double)dk * (double)cL[f];
  }
  if (act && t == 0) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      sh_line[lil][f][1] = (double)AR[f] + (double)m * (double)cR[f];
      sh_line[lil][f][2] = (double)seg.jln[f];
    }
  }
  __syncthreads();
  // the FP64 2x2 boundary solve, once per line
  if (act && t < F) {
    double Ba, Bb;
    boundary_terms(c, sh_line[lil][t][0], sh_line[lil][t][1], sh_line[lil][t][2], Ba, Bb);
    sh_line[lil][t][0] = Ba;
    sh_line[lil][t][1] = Bb;
  }
  __syncthreads();

  // phase C: seeded scans; the swept values go back to LDS (every read of the
  // window happened before the barriers of the carry scan above)
  if (has) {
    const int jlast = min(j0 + K - 1, n - 1);
    const T pL = dpow<T>(c.nu, (double)j0);
    const T pR = dpow<T>(c.nu, (double)(c.N - jlast));
    T gL[F], gR[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      gL[f] = d * cL[f] + (T)(2.0 * sh_line[lil][f][0]) * pL;
      gR[f] = d * cR[f] + (T)(2.0 * sh_line[lil][f][1]) * pR;
    }
    T w[F][K];
    seg.finalize(d, j0, n, gL, gR, w);
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (j0 + k < n) {
#pragma unroll
        for (int f = 0; f < F; ++f) sh_row[f][MOLT_PAD(rowoff + j0 + k)] = w[f][k];
      }
  }
  __syncthreads();

  // phase D: outputs in the coalesced layout of phase A
  double resid = 0.0;
  if (act) {
    if (vec) {
#pragma unroll
      for (int it = 0; it < K / V; ++it) {
        const int e0 = (it * TL + t) * V;
        if (e0 < n) {
          T o[NO][V];
          T lv[LT > 0 ? LT : 1][V];
#pragma unroll
          for (int l = 0; l < LT; ++l) ld16((const T*)a.in[NR + l] + lbase + (size_t)e0, lv[l]);
#pragma unroll
          for (int v = 0; v < V; ++v) {
            T wk[F], xk[E + LT > 0 ? E + LT : 1], ok[NO];
#pragma unroll
            for (int f = 0; f < F; ++f) wk[f] = sh_row[f][MOLT_PAD(rowoff + e0 + v)];
#pragma unroll
            for (int e = 0; e < E; ++e) xk[e] = seg.ex[e][it * V + v];
#pragma unroll
            for (int l = 0; l < LT; ++l) xk[E + l] = lv[l][v];
            resid = fmax(resid, P::fin(a, wk, xk, ok));
#pragma unroll
            for (int f = 0; f < NO; ++f) o[f][v] = ok[f];
          }
#pragma unroll
          for (int f = 0; f < NO; ++f) st16_prog<T, P>(a, f, lbase + (size_t)e0, o[f]);
        }
      }
    } else {
#pragma unroll
      for (int it = 0; it < K; ++it) {
        const int e = it * TL + t;
        if (e < n) {
          T wk[F], xk[E + LT > 0 ? E + LT : 1], ok[NO];
#pragma unroll
          for (int f = 0; f < F; ++f) wk[f] = sh_row[f][MOLT_PAD(rowoff + e)];
#pragma unroll
          for (int q = 0; q < E; ++q) xk[q] = seg.ex[q][it];
#pragma unroll
          for (int l = 0; l < LT; ++l) xk[E + l] = ((const T*)a.in[NR + l])[lbase + (size_t)e];
          resid = fmax(resid, P::fin(a, wk, xk, ok));
#pragma unroll
          for (int f = 0; f < NO; ++f) st1_prog<T, P>(a, f, lbase + (size_t)e, ok[f]);
        }
      }
    }
  }
#undef MOLT_PAD
  if (rpart != nullptr) residual_block(resid, rpart, bx);
}


// --------------------------------------------------------------------------
// y-direction pass.  Block = 64 consecutive columns (one wave wide: every row
// access is a coalesced 64-element segment) x RG thread rows; thread (col, t)
// owns rows t*K .. t*K+K-1 of its column.  Three kernels:
//  ytot: zero-seeded totals per thread -> tot[f][dir][t][col]
//  ycomb: per column, FP64 exclusive scans over threads, line totals, the
//         boundary solve and the seeds, written over tot
//  yfin: seeded scans and the program outputs
// --------------------------------------------------------------------------

template <typename T, int PI, int K, int M, bool PER>
__device__ __forceinline__ void ytot_body(const LineCoef& c, const PassArgs& a, DevState* st, int nx, int nth,
                                          int nseg, size_t fstride, T* agg, T* jlnb, int bx, int by, int bz) {
  using P = typename ProgOf<PI, T>::type;
  constexpr int F = P::F;
  if (st != nullptr && st->done) return;
  __shared__ T shA[F][2][kRG][64];
  const int lx = threadIdx.x, r = threadIdx.y;
  const int col = bx * 64 + lx;
  const int sg = by;
  const int t = sg * kRG + r;
  const int b = bz;
  const bool ok = col < nx && t < nth;
  const int n = c.n, j0 = t * K;
  const size_t lbase = (size_t)b * fstride + (size_t)(col < nx ? col : 0);
  T AL[F], AR[F];
  if (ok) {
    Seg<T, P, K, M, PER> seg;
    seg.build(c, a, lbase, (size_t)nx, j0, false);
    seg.totals((T)c.d, j0, n, AL, AR);
    if (t == 0) {
#pragma unroll
      for (int f = 0; f < F; ++f) jlnb[((size_t)b * F + f) * nx + col] = seg.jln[f];
    }
  } else {
#pragma unroll
    for (int f = 0; f < F; ++f) AL[f] = AR[f] = T(0);
  }
#pragma unroll
  for (int f = 0; f < F; ++f) {
    shA[f][0][r][lx] = AL[f];
    shA[f][1][r][lx] = AR[f];
  }
  __syncthreads();
  if (r != 0 || col >= nx) return;
  // the segment's zero-seeded totals: L at its last row, R at its first row
  const int j0s = sg * kRG * K;
  const int jls = min(j0s + kRG * K - 1, n - 1);
  T* ab = agg + (size_t)b * (size_t)(F * 2) * nseg * nx;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    T L = T(0), R = T(0);
#pragma unroll
    for (int g = 0; g < kRG; ++g) {
      const int tt = sg * kRG + g;
      if (tt < nth) {
        const int jl = min(tt * K + K - 1, n - 1);
        L += dpow<T>(c.nu, (double)(jls - jl)) * shA[f][0][g][lx];
        R += dpow<T>(c.nu, (double)(tt * K - j0s)) * shA[f][1][g][lx];
      }
    }
    ab[((size_t)(f * 2 + 0) * nseg + sg) * nx + col] = L;
    ab[((size_t)(f * 2 + 1) * nseg + sg) * nx + col] = R;
  }
}


// yloc: the deferred y-pass in one read of its inputs.  Each segment of
// kRG*K rows is scanned from zero (block-internal carries through LDS), the
// program's outputs are written from these segment-local values, and the
// segment's zero-seeded totals (and the periodic closing quadrature) go to agg
// / jlnb for ycomb, whose seeds the next x-pass adds (YCorr).
template <typename T, int PI, int K, int M, bool PER>
__device__ __forceinline__ void yloc_body(const LineCoef& c, const PassArgs& a, DevState* st, int nx, int nth,
                                          int nseg, size_t fstride, T* agg, T* jlnb, int bx, int by, int bz) {
  using P = typename ProgOf<PI, T>::type;
  constexpr int F = P::F;
  // P1 of an iteration: its first block closes the previous iteration (the
  // other blocks may still see done = 0 and compute this pass's temporaries,
  // which the next passes, seeing the close, then leave unused)
  if (a.close_part != nullptr && bx == 0 && by == 0 && bz == 0) {
    if (residual_close_pending(a.close_part, st)) return;
  } else if (st != nullptr && st->done) {
    return;
  }
  __shared__ T shA[F][2][kRG][64];
  const int lx = threadIdx.x, r = threadIdx.y;
  const int col = bx * 64 + lx;
  const int sg = by;
  const int t = sg * kRG + r;
  const int b = bz;
  const bool ok = col < nx && t < nth;
  const int n = c.n, j0 = t * K;
  const size_t lbase = (size_t)b * fstride + (size_t)(col < nx ? col : 0);
  const T d = (T)c.d;
  Seg<T, P, K, M, PER> seg;
  T AL[F], AR[F];
  if (ok) {
    seg.build(c, a, lbase, (size_t)nx, j0, false);
    seg.totals(d, j0, n, AL, AR);
    if (t == 0) {
#pragma unroll
      for (int f = 0; f < F; ++f) jlnb[((size_t)b * F + f) * nx + col] = seg.jln[f];
    }
  } else {
#pragma unroll
    for (int f = 0; f < F; ++f) AL[f] = AR[f] = T(0);
  }
#pragma unroll
  for (int f = 0; f < F; ++f) {
    shA[f][0][r][lx] = AL[f];
    shA[f][1][r][lx] = AR[f];
  }
  __syncthreads();
  const int j0s = sg * kRG * K;
  const int jls = min(j0s + kRG * K - 1, n - 1);
  if (r == 0 && col < nx) {
    // the segment's zero-seeded totals: L at its last row, R at its first row
    T* ab = agg + (size_t)b * (size_t)(F * 2) * nseg * nx;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      T L = T(0), R = T(0);
#pragma unroll
      for (int g = 0; g < kRG; ++g) {
        const int tt = sg * kRG + g;
        if (tt < nth) {
          const int jl = min(tt * K + K - 1, n - 1);
          L += dpow<T>(c.nu, (double)(jls - jl)) * shA[f][0][g][lx];
          R += dpow<T>(c.nu, (double)(tt * K - j0s)) * shA[f][1][g][lx];
        }
      }
      ab[((size_t)(f * 2 + 0) * nseg + sg) * nx + col] = L;
      ab[((size_t)(f * 2 + 1) * nseg + sg) * nx + col] = R;
    }
  }
  if (!ok) return;
  // carries from the segment's other thread rows only (the segment starts
  // from zero at both ends)
  const T mK = dpow<T>(c.nu, (double)K);
  T gL[F], gR[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    T cl = T(0), cr = T(0);
    for (int g = 0; g < r; ++g) cl = mK * cl + shA[f][0][g][lx];
    for (int g = kRG - 1; g > r; --g)
      if (sg * kRG + g < nth) cr = mK * cr + shA[f][1][g][lx];
    gL[f] = d * cl;
    gR[f] = d * cr;
  }
  T w[F][K];
  seg.finalize(d, j0, n, gL, gR, w);
  seg.store(a, lbase, (size_t)nx, j0, n, false, w);
}


// ycomb: one block = 64 columns x 16 waves for one field of one batch entry.
// Wave w owns threads [w*CT, w*CT + CT) of every column (CT = ceil(nth/16) <=
// CTMAX): chunk-local scans, chunk carries through LDS, then the line totals,
// the FP64 boundary solve and the seeds, written over the totals.
constexpr int kCombWaves = 16;

template <typename T, int CTMAX>
__device__ __forceinline__ void ycomb_body(const LineCoef& c, DevState* st, int nx, int nth, int K, int F, T* tot,
                                           const T* jlnb, int bx, int by, int bz) {
  if (st != nullptr && st->done) return;
  __shared__ double shL[kCombWaves][64], shR[kCombWaves][64];
  __shared__ double shTL[64], shTR[64];
  const int lane = threadIdx.x, w = threadIdx.y;
  const int col = bx * 64 + lane;
  const int f = by, b = bz;
  const bool ok = col < nx;
  const int n = c.n;
  const int CT = (nth + kCombWaves - 1) / kCombWaves;
  const int t0 = w * CT;
  T* tb = tot + (size_t)b * (size_t)(F * 2) * nth * nx;
  T* AL = tb + (size_t)(f * 2 + 0) * nth * nx + (ok ? col : 0);
  T* AR = tb + (size_t)(f * 2 + 1) * nth * nx + (ok ? col : 0);
  const double d = c.d, nu = c.nu;
  const double m = exp(-nu * (double)K), mC = exp(-nu * (double)K * (double)CT);
  T vL[CTMAX], vR[CTMAX];
#pragma unroll
  for (int i = 0; i < CTMAX; ++i) {
    const int t = t0 + i;
    const bool in = ok && i < CT && t < nth;
    vL[i] = in ? AL[(size_t)t * nx] : T(0);
    vR[i] = in ? AR[(size_t)t * nx] : T(0);
  }
  // chunk totals over the chunk's own entries (entries past nth are zero)
  double xl = 0.0, xr = 0.0;
#pragma unroll
  for (int i = 0; i < CTMAX; ++i)
    if (i < CT) xl = m * xl + (double)vL[i];
#pragma unroll
  for (int i = CTMAX - 1; i >= 0; --i) xr = m * xr + (double)vR[i];
  shL[w][lane] = xl;
  shR[w][lane] = xr;
  __syncthreads();
  double CL = 0.0, CR = 0.0;
  for (int v = 0; v < w; ++v) CL = mC * CL + shL[v][lane];
  for (int v = kCombWaves - 1; v > w; --v) CR = mC * CR + shR[v][lane];
  const int tstar = (n - 1) / K;
  const double dk = exp(-nu * (double)(n - 1 - tstar * K + 1));
  double cl = CL;
#pragma unroll
  for (int i = 0; i < CTMAX; ++i) {
    const int t = t0 + i;
    const double v = (double)vL[i];
    if (i < CT && t == tstar) shTL[lane] = v + dk * cl;
    vL[i] = (T)cl;  // exclusive carry into thread t
    cl = m * cl + v;
  }
  double cr = CR;
#pragma unroll
  for (int i = CTMAX - 1; i >= 0; --i) {
    if (i < CT) {  // entries past the chunk must not decay the carry
      const int t = t0 + i;
      const double v = (double)vR[i];
      if (t == 0) shTR[lane] = v + m * cr;
      vR[i] = (T)cr;
      cr = m * cr + v;
    }
  }
  __syncthreads();
  if (!ok) return;
  double Ba, Bb;
  boundary_terms(c, shTL[lane], shTR[lane], (double)jlnb[((size_t)b * F + f) * nx + col], Ba, Bb);
  double pL = exp(-nu * (double)t0 * (double)K);
#pragma unroll
  for (int i = 0; i < CTMAX; ++i) {
    const int t = t0 + i;
    if (i < CT && t < nth) AL[(size_t)t * nx] = (T)(d * (double)vL[i] + 2.0 * Ba * pL);
    pL *= m;
  }
  double pR = 0.0;
  bool first = true;
#pragma unroll
  for (int i = CTMAX - 1; i >= 0; --i) {
    const int t = t0 + i;
    if (i < CT && t < nth) {
      const int jlast = min(t * K + K - 1, n - 1);
      pR = (first || t >= nth - 2) ? exp(-nu * (double)(c.N - jlast)) : pR * m;
      first = false;
      AR[(size_t)t * nx] = (T)(d * (double)vR[i] + 2.0 * Bb * pR);
    }
  }
}


template <typename T, int PI, int K, int M, bool PER>
__device__ __forceinline__ void yfin_body(const LineCoef& c, const PassArgs& a, DevState* st, int nx, int nth,
                                          int nseg, size_t fstride, const T* seeds, int bx, int by, int bz) {
  using P = typename ProgOf<PI, T>::type;
  constexpr int F = P::F;
  if (st != nullptr && st->done) return;
  __shared__ T shA[F][2][kRG][64];
  const int lx = threadIdx.x, r = threadIdx.y;
  const int col = bx * 64 + lx;
  const int sg = by;
  const int t = sg * kRG + r;
  const int b = bz;
  const bool ok = col < nx && t < nth;
  const int n = c.n, j0 = t * K;
  const size_t lbase = (size_t)b * fstride + (size_t)(col < nx ? col : 0);
  const T d = (T)c.d;
  Seg<T, P, K, M, PER> seg;
  T AL[F], AR[F];
  if (ok) {
    seg.build(c, a, lbase, (size_t)nx, j0, false);
    seg.totals(d, j0, n, AL, AR);
  } else {
#pragma unroll
    for (int f = 0; f < F; ++f) AL[f] = AR[f] = T(0);
  }
#pragma unroll
  for (int f = 0; f < F; ++f) {
    shA[f][0][r][lx] = AL[f];
    shA[f][1][r][lx] = AR[f];
  }
  __syncthreads();
  if (!ok) return;
  // carries from the other thread rows of the segment (all rows before a
  // thread with nodes are full, rows after it start K apart), then the
  // segment's seeds propagated to this thread's first / last node
  const T mK = dpow<T>(c.nu, (double)K);
  const int j0s = sg * kRG * K;
  const int jls = min(j0s + kRG * K - 1, n - 1);
  const int jlt = min(j0 + K - 1, n - 1);
  const T* sb = seeds + (size_t)b * (size_t)(F * 2) * nseg * nx;
  const T pl = dpow<T>(c.nu, (double)(j0 - j0s)), pr = dpow<T>(c.nu, (double)(jls - jlt));
  T gL[F], gR[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    T cl = T(0), cr = T(0);
    for (int g = 0; g < r; ++g) cl = mK * cl + shA[f][0][g][lx];
    for (int g = kRG - 1; g > r; --g)
      if (sg * kRG + g < nth) cr = mK * cr + shA[f][1][g][lx];
    gL[f] = d * cl + pl * sb[((size_t)(f * 2 + 0) * nseg + sg) * nx + col];
    gR[f] = d * cr + pr * sb[((size_t)(f * 2 + 1) * nseg + sg) * nx + col];
  }
  T w[F][K];
  seg.finalize(d, j0, n, gL, gR, w);
  seg.store(a, lbase, (size_t)nx, j0, n, false, w);
}

// FP64 mass and energy partial sums (fixed grid, fixed order: deterministic).
// Block bx takes rows bx, bx + nb, ...; its threads stride along the row.
template <typename T>
__device__ __forceinline__ void diag_body(const T* u, int nx, int ny, int bc, double hx, double hy, double eps,
                                          double* partials, int bx, int nb) {
  __shared__ double sm[2][4];
  const bool per = bc == MOLT_BC_PERIODIC;
  const double ihx = 1.0 / hx, ihy = 1.0 / hy, ge = 0.5 * eps * eps;
  double ms = 0.0, en = 0.0;
  for (int iy = bx; iy < ny; iy += nb) {
    const double wy = (ny == 1 || per) ? 1.0 : ((iy == 0 || iy == ny - 1) ? 0.5 : 1.0);
    const T* row = u + (size_t)iy * nx;
    const T* up = u + (size_t)(iy + 1 == ny ? 0 : iy + 1) * nx;
    const bool gy = ny > 1 && (per || iy < ny - 1);
    // four nodes per thread and pass, all loads issued before the sums
    for (int x0 = threadIdx.x; x0 < nx; x0 += 4 * blockDim.x) {
      T c0[4], c1[4], c2[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ix = min(x0 + q * (int)blockDim.x, nx - 1);
        c0[q] = row[ix];
        c1[q] = row[ix + 1 == nx ? 0 : ix + 1];
        c2[q] = up[ix];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ix = x0 + q * (int)blockDim.x;
        if (ix >= nx) break;
        const double wx = per ? 1.0 : ((ix == 0 || ix == nx - 1) ? 0.5 : 1.0);
        const double uu = (double)c0[q];
        ms += wx * wy * uu;
        const double qq = uu * uu - 1.0;
        en += wx * wy * 0.25 * qq * qq;
        if (per || ix < nx - 1) {
          const double g = ((double)c1[q] - uu) * ihx;
          en += ge * g * g * wy;
        }
        if (gy) {
          const double g = ((double)c2[q] - uu) * ihy;
          en += ge * g * g * wx;
        }
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ms += __shfl_down(ms, off);
    en += __shfl_down(en, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sm[0][wave] = ms;
    sm[1][wave] = en;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 4; ++w) {
      a += sm[0][w];
      b += sm[1][w];
    }
    partials[2 * bx] = a;
    partials[2 * bx + 1] = b;
  }
}

// max |a - b| over n elements (FP64, order independent): one partial per block
template <typename T>
__device__ __forceinline__ void maxdiff_body(const T* a, const T* b, size_t n, double* partials, int bx, int nb) {
  __shared__ double sm[4];
  double m = 0.0;
  for (size_t i = (size_t)bx * blockDim.x + threadIdx.x; i < n; i += (size_t)nb * blockDim.x)
    m = fmax(m, fabs((double)a[i] - (double)b[i]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) partials[bx] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
}

// mass and energy of the field from the per-block partial sums
__device__ __forceinline__ void diag_final_body(const double* partials, int nblocks, double area, DevState* st) {
  __shared__ double sm[2][256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  sm[0][threadIdx.x] = a;
  sm[1][threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + s];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->mass = sm[0][0] * area;
    st->energy = sm[1][0] * area;
  }
}

// --------------------------------------------------------------------------
// Vector model (Sec. 2 eq. CH_vector_reaction, Sec. 5.2).  With w = u1 + i u2,
// prod_i |u - z_i|^2 over the cube roots of unity is |w^3 - 1|^2, so
// grad W = (Re G, Im G) with G = 2 dW/d(conj w) = 6 conj(w)^2 (w^3 - 1)
//        = 6 (|w|^4 w - conj(w)^2).
// In u the shifted reaction g(v) = grad W(v + z3) - sigma v is
// grad W(u) - sigma u up to a constant, which C1 annihilates.
//  full form:      e = G(p) - sigma p, lin = p
//  increment form: e = G(p) - G(q) - sigma d, lin = d  (p = q + d), with
//    G(p) - G(q) = 6 [ |p|^4 d + (|p|^2 - |q|^2)(|p|^2 + |q|^2) q - conj(d) conj(p + q) ],
//    |p|^2 - |q|^2 = Re(d conj(p + q)): every term is proportional to d, so an
//    FP32 increment keeps its relative accuracy.
// --------------------------------------------------------------------------
// (c1, c2): u = stored value + c; 0 when the fields hold u, z3 when they hold
// the shifted variable v = u - z3 (Dirichlet steps)
template <typename T>
__device__ __forceinline__ void vch_react(T b1, T b2, T w1, T w2, T d1, T d2, T c1u, T c2u, T sigma, int mode,
                                          T* e, T* lin) {
#pragma clang fp contract(off)
  if (mode == 0) {
    const T u1 = b1 + c1u, u2 = b2 + c2u;
    const T p2 = u1 * u1 + u2 * u2;
    const T p4 = p2 * p2;
    // conj(w)^2 = (u1^2 - u2^2, -2 u1 u2)
    e[0] = T(6) * (p4 * u1 - (u1 * u1 - u2 * u2)) - sigma * b1;
    e[1] = T(6) * (p4 * u2 + T(2) * u1 * u2) - sigma * b2;
    lin[0] = b1;
    lin[1] = b2;
  } else {
    const T p1 = b1 + c1u + w1, p2c = b2 + c2u + w2;  // current iterate p (in u)
    const T q1 = p1 - d1, q2 = p2c - d2;  // previous iterate q
    const T s1 = p1 + q1, s2 = p2c + q2;
    const T P2 = p1 * p1 + p2c * p2c, Q2 = q1 * q1 + q2 * q2;
    const T dr = d1 * s1 + d2 * s2;  // |p|^2 - |q|^2
    const T tq = dr * (P2 + Q2);      // |p|^4 - |q|^4
    const T P4 = P2 * P2;
    // conj(d) conj(s) = conj(d s) = (d1 s1 - d2 s2, -(d1 s2 + d2 s1))
    const T c1 = d1 * s1 - d2 * s2, c2 = -(d1 * s2 + d2 * s1);
    e[0] = T(6) * (P4 * d1 + tq * q1 - c1) - sigma * d1;
    e[1] = T(6) * (P4 * d2 + tq * q2 - c2) - sigma * d2;
    lin[0] = d1;
    lin[1] = d2;
  }
}

// (e, lin) of both components at nodes [i0, n) with stride `step`: in = (base,
// W, dl), out = (e, lin), every field component-major with n nodes per component
template <typename T>
__device__ __forceinline__ void vch_react_body(const PassArgs& a, size_t n, size_t i0, size_t step) {
  const T* B = (const T*)a.in[0];
  const T* Wf = (const T*)a.in[1];
  const T* D = (const T*)a.in[2];
  T* E = (T*)a.out[0];
  T* L = (T*)a.out[1];
  const T sg = (T)a.sigma;
  const T c1 = (T)a.ushift[0], c2 = (T)a.ushift[1];
  for (size_t i = i0; i < n; i += step) {
    T e[2], lin[2];
    if (a.mode == 0)
      vch_react<T>(B[i], B[n + i], T(0), T(0), T(0), T(0), c1, c2, sg, 0, e, lin);
    else
      vch_react<T>(B[i], B[n + i], Wf[i], Wf[n + i], D[i], D[n + i], c1, c2, sg, 1, e, lin);
    E[i] = e[0];
    E[n + i] = e[1];
    L[i] = lin[0];
    L[n + i] = lin[1];
  }
}

// FP64 mass of each component and the energy of eq. EnergyFunctional_vector
// (forward differences, trapezoid end weights off the periodic case); three
// partial sums per block
template <typename T>
__device__ __forceinline__ void diag_vch_body(const T* u, int nx, int ny, int bc, double hx, double hy, double eps,
                                              double* partials, int bx, int nb) {
  __shared__ double sm[3][4];
  const bool per = bc == MOLT_BC_PERIODIC;
  const double ihx = 1.0 / hx, ihy = 1.0 / hy, ge = 0.5 * eps * eps;
  double m1 = 0.0, m2 = 0.0, en = 0.0;
  const size_t n = (size_t)nx * ny;
  for (int iy = bx; iy < ny; iy += nb) {
    const double wy = (ny == 1 || per) ? 1.0 : ((iy == 0 || iy == ny - 1) ? 0.5 : 1.0);
    const size_t r0 = (size_t)iy * nx, r1 = (size_t)(iy + 1 == ny ? 0 : iy + 1) * nx;
    const bool gy = ny > 1 && (per || iy < ny - 1);
#pragma unroll 2
    for (int ix = threadIdx.x; ix < nx; ix += blockDim.x) {
      const double wx = per ? 1.0 : ((ix == 0 || ix == nx - 1) ? 0.5 : 1.0);
      const size_t i = r0 + ix;
      const double a = (double)u[i], b = (double)u[n + i];
      m1 += wx * wy * a;
      m2 += wx * wy * b;
      // |w^3 - 1|^2 with w^3 = (a^3 - 3ab^2, 3a^2 b - b^3)
      const double r = a * a * a - 3.0 * a * b * b - 1.0, s = 3.0 * a * a * b - b * b * b;
      en += wx * wy * (r * r + s * s);
      for (int c = 0; c < 2; ++c) {
        const T* uc = u + c * n;
        const double uu = (double)uc[i];
        if (per || ix < nx - 1) {
          const double g = ((double)uc[r0 + (ix + 1 == nx ? 0 : ix + 1)] - uu) * ihx;
          en += ge * g * g * wy;
        }
        if (gy) {
          const double g = ((double)uc[r1 + ix] - uu) * ihy;
          en += ge * g * g * wx;
        }
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m1 += __shfl_down(m1, off);
    m2 += __shfl_down(m2, off);
    en += __shfl_down(en, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sm[0][wave] = m1;
    sm[1][wave] = m2;
    sm[2][wave] = en;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0, y = 0.0, z = 0.0;
    for (int w = 0; w < 4; ++w) {
      x += sm[0][w];
      y += sm[1][w];
      z += sm[2][w];
    }
    partials[3 * bx] = x;
    partials[3 * bx + 1] = y;
    partials[3 * bx + 2] = z;
  }
}

__device__ __forceinline__ void diag_vch_final_body(const double* partials, int nblocks, double area, DevState* st) {
  __shared__ double sm[3][256];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
    a += partials[3 * i];
    b += partials[3 * i + 1];
    c += partials[3 * i + 2];
  }
  sm[0][threadIdx.x] = a;
  sm[1][threadIdx.x] = b;
  sm[2][threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + s];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
      sm[2][threadIdx.x] += sm[2][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->mass = sm[0][0] * area;
    st->mass2 = sm[1][0] * area;
    st->energy = sm[2][0] * area;
  }
}

}  // namespace molt
