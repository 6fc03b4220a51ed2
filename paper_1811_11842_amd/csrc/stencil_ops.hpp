// Pointwise stencil arithmetic shared by the plain and the streaming kernels:
// the 5-point Laplacian (OP 0), the 13-point Cahn-Hilliard operator (OP 1)
// and the 5-point Helmholtz operator of the momentum predictor (OP 2) on
// values already gathered, in float64 and in double-double (error-free
// transforms).
//
// OP 2, x + s (4 x - axis neighbours) with s = beta n^2, has Dirichlet walls:
// its rows 0 and n are identity rows (the wall value is data), which the
// callers realise with a zero coefficient there (row_coef) and a zero
// smoother weight (row_dinv), so iterates and corrections never change the
// wall rows; the first and last interior rows read the wall rows as they are.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace bf {

// Values around one node: centre c; axis neighbours at distance 1 (x-1, x+1,
// y-1, y+1); diagonals; axis neighbours at distance 2.  Ghost rows are
// already reflected and columns wrapped by the caller.  T is the storage and
// arithmetic type (double, or float inside the mixed-precision V-cycle).
template <typename T>
struct Nb13T {
  T c;
  T xm1, xp1, ym1, yp1;
  T dmm, dmp, dpm, dpp;  // (y-1,x-1) (y-1,x+1) (y+1,x-1) (y+1,x+1)
  T xm2, xp2, ym2, yp2;
};
using Nb13 = Nb13T<double>;

// Gather the stencil values around (i, j) of an (n+1) x n field at x (global
// or LDS): ghost rows reflected, columns wrapped.
template <int OP, typename T>
__device__ __forceinline__ Nb13T<T> gather(const T* x, int i, int j, int n, int mask) {
  Nb13T<T> v;
  const T* r0 = x + (int64_t)j * n;
  const T* rm1 = x + (int64_t)refl(j - 1, n) * n;
  const T* rp1 = x + (int64_t)refl(j + 1, n) * n;
  const int im1 = (i - 1) & mask, ip1 = (i + 1) & mask;
  v.c = r0[i];
  v.xm1 = r0[im1];
  v.xp1 = r0[ip1];
  v.ym1 = rm1[i];
  v.yp1 = rp1[i];
  if (OP == 1) {
    const T* rm2 = x + (int64_t)refl(j - 2, n) * n;
    const T* rp2 = x + (int64_t)refl(j + 2, n) * n;
    const int im2 = (i - 2) & mask, ip2 = (i + 2) & mask;
    v.dmm = rm1[im1];
    v.dmp = rm1[ip1];
    v.dpm = rp1[im1];
    v.dpp = rp1[ip1];
    v.xm2 = r0[im2];
    v.xp2 = r0[ip2];
    v.ym2 = rm2[i];
    v.yp2 = rp2[i];
  }
  return v;
}

// coarse(J, I) = sum_{dj, di in {0, +-1, +-3}} w_dj w_di fine(2J+dj, 2I+di),
// w_0 = 1/2, w_{+-1} = 9/32, w_{+-3} = -1/32 (the weighted adjoint of cubic
// interpolation, scaled by 1/4); fine rows reflected, columns wrapped.
template <typename T>
__device__ __forceinline__ T restrict_at(const T* fine, int nf, int fmask, int I, int J) {
  const int off[5] = {-3, -1, 0, 1, 3};
  const T w[5] = {T(-1.0 / 32), T(9.0 / 32), T(0.5), T(9.0 / 32), T(-1.0 / 32)};
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    const T* row = fine + (int64_t)refl(2 * J + off[a], nf) * nf;
    T rs = T(0);
#pragma unroll
    for (int c = 0; c < 5; ++c) rs += w[c] * row[(2 * I + off[c]) & fmask];
    acc += w[a] * rs;
  }
  return acc;
}

// (P coarse)(j, i): tensor-product cubic interpolation (-1, 9, 9, -1)/16 at
// odd fine nodes, injection at even ones; coarse rows reflected, columns wrapped.
template <typename T>
__device__ __forceinline__ T interp_x_at(const T* coarse, int nc, int cmask, int J, int i) {
  const T* row = coarse + (int64_t)refl(J, nc) * nc;
  const int I = i >> 1;
  if ((i & 1) == 0) return row[I];
  return (-row[(I - 1) & cmask] + T(9) * row[I] + T(9) * row[(I + 1) & cmask] -
          row[(I + 2) & cmask]) *
         T(0.0625);
}

template <typename T>
__device__ __forceinline__ T prolong_at(const T* coarse, int nc, int cmask, int i, int j) {
  const int J = j >> 1;
  if ((j & 1) == 0) return interp_x_at(coarse, nc, cmask, J, i);
  return (-interp_x_at(coarse, nc, cmask, J - 1, i) + T(9) * interp_x_at(coarse, nc, cmask, J, i) +
          T(9) * interp_x_at(coarse, nc, cmask, J + 1, i) -
          interp_x_at(coarse, nc, cmask, J + 2, i)) *
         T(0.0625);
}

// Coefficient of the stencil term on row j (OP 2: 0 on the wall rows, which
// makes them identity rows).
template <int OP>
__host__ __device__ __forceinline__ double row_coef(double coef, int j, int n) {
  return (OP == 2 && (j == 0 || j == n)) ? 0.0 : coef;
}

// Smoother weight D^{-1} on row j: the 13-point operator's diagonal is 21 s
// on rows 1 and n-1 (dinv_edge there); OP 2 leaves its wall rows alone
// (dinv_edge = 0 there).
template <int OP, typename R = double>
__host__ __device__ __forceinline__ R row_dinv(R dinv_int, R dinv_edge, int j, int n) {
  if (OP == 1) return (j == 1 || j == n - 1) ? dinv_edge : dinv_int;
  if (OP == 2) return (j == 0 || j == n) ? dinv_edge : dinv_int;
  return dinv_int;
}

// A x at the node.  OP 0: n^2 (axis - 4 c); OP 1: c + s (20 c - 8 axis + 2 diag + far);
// OP 2: c + s (4 c - axis).
template <int OP, typename T>
__device__ __forceinline__ T apply_vals(const Nb13T<T>& v, T coef) {
  const T axis = (v.xm1 + v.xp1) + (v.ym1 + v.yp1);
  if (OP == 0) return coef * (axis - T(4) * v.c);
  if (OP == 2) return v.c + coef * (T(4) * v.c - axis);
  const T diag = (v.dmm + v.dmp) + (v.dpm + v.dpp);
  const T far = (v.xm2 + v.xp2) + (v.ym2 + v.yp2);
  return v.c + coef * (T(20) * v.c - T(8) * axis + T(2) * diag + far);
}

// Error-free transformations (Knuth TwoSum; TwoProduct through fma).  They
// rely on every product and sum being rounded separately, so floating-point
// contraction (fusing a*b + c into one fma, which hipcc does by default) is
// switched off inside them and inside their callers.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
#pragma clang fp contract(off)
  p = a * b;
  e = fma(a, b, -p);
}

// Double-double numbers (hi + lo, |lo| <= ulp(hi)/2) for the variable-
// mobility operator, whose coefficients are not small integers: sums and
// products by float64 values carried with the error-free transformations
// above (Dekker/Knuth; relative error of a few u^2).
struct DD {
  double hi, lo;
};

__device__ __forceinline__ DD dd_norm(double s, double e) {
#pragma clang fp contract(off)
  const double hi = s + e;
  return DD{hi, e - (hi - s)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b) {
#pragma clang fp contract(off)
  double s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  return dd_norm(s, e);
}

__device__ __forceinline__ DD dd_add_d(DD a, double b) {
#pragma clang fp contract(off)
  double s, e;
  two_sum(a.hi, b, s, e);
  e += a.lo;
  return dd_norm(s, e);
}

__device__ __forceinline__ DD dd_sub(DD a, DD b) { return dd_add(a, DD{-b.hi, -b.lo}); }

__device__ __forceinline__ DD dd_mul_d(DD a, double b) {
#pragma clang fp contract(off)
  double p, e;
  two_prod(a.hi, b, p, e);
  e = fma(a.lo, b, e);
  return dd_norm(p, e);
}

// (a + b + c + d - 4 e) as a double-double (Sum2 cascade; 4 e is exact).
__device__ __forceinline__ DD dd_lap_sum(double a, double b, double c, double d, double e) {
#pragma clang fp contract(off)
  const double t[4] = {b, c, d, -4.0 * e};
  double hi = a, lo = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double err;
    two_sum(hi, t[k], hi, err);
    lo += err;
  }
  return dd_norm(hi, lo);
}

// b - A x with the stencil sum carried in double-double: the integer stencil
// weights make every term exact (20 c through two_prod, the others are
// power-of-two multiples), the cascaded two_sum (Ogita-Rump-Oishi Sum2)
// returns the sum as if computed in twice the working precision, and the
// scaling by s = c n^4 (or n^2) is a two_prod.  The result is accurate to a
// few ulps of itself instead of u * (c/h^4) * |x|.
template <int OP>
__device__ __forceinline__ double residual_dd_vals(const Nb13& v, double bval, double coef) {
#pragma clang fp contract(off)
  double t[14];
  int nt;
  if (OP == 0) {
    t[0] = v.xm1; t[1] = v.xp1; t[2] = v.ym1; t[3] = v.yp1; t[4] = -4.0 * v.c;
    nt = 5;
  } else if (OP == 2) {
    t[0] = 4.0 * v.c; t[1] = -v.xm1; t[2] = -v.xp1; t[3] = -v.ym1; t[4] = -v.yp1;
    nt = 5;
  } else {
    two_prod(20.0, v.c, t[0], t[1]);
    t[2] = -8.0 * v.xm1; t[3] = -8.0 * v.xp1; t[4] = -8.0 * v.ym1; t[5] = -8.0 * v.yp1;
    t[6] = 2.0 * v.dmm; t[7] = 2.0 * v.dmp; t[8] = 2.0 * v.dpm; t[9] = 2.0 * v.dpp;
    t[10] = v.xm2; t[11] = v.xp2; t[12] = v.ym2; t[13] = v.yp2;
    nt = 14;
  }
  double hi = t[0], lo = 0.0;
#pragma unroll
  for (int k = 1; k < 14; ++k) {
    if (k < nt) {
      double e;
      two_sum(hi, t[k], hi, e);
      lo += e;
    }
  }
  double ph, pe;
  two_prod(coef, hi, ph, pe);
  pe = fma(coef, lo, pe);
  double w, ve = pe;
  if (OP != 0) {
    double e;
    two_sum(v.c, ph, w, e);
    ve = pe + e;
  } else {
    w = ph;
  }
  double r, re;
  two_sum(bval, -w, r, re);
  return r + (re - ve);
}

// Exact 13-point operator by splitting (the ExtractScalar step of Rump, Ogita
// and Oishi's accurate summation).  With sigma a power of two that bounds 64
// times every value the stencil combines, hi = fl(fl(sigma + v) - sigma) is a
// multiple of u sigma (u = 2^-53) and lo = v - hi is exact with |lo| <= u
// sigma.  The integer-weighted sum of the hi parts (weights 20, -8, 2, 1,
// sum of |weights| 64) is then a multiple of u sigma of magnitude below sigma,
// so every partial sum is representable and the float64 sum is exact in any
// order; the lo parts sum with an absolute error of a few u^2 sigma.  The
// split is done once per value of a wavefront's window (shared by all the
// stencils that read it) instead of one compensated step per stencil term.
__device__ __forceinline__ void split_sigma(double v, double sigma, double& hi, double& lo) {
#pragma clang fp contract(off)
  hi = (sigma + v) - sigma;
  lo = v - hi;
}

// q = c + s * S13(v) from the split neighbourhoods vh (hi parts, centre vh.c)
// and vl (lo parts), c = vh.c + vl.c (exact): the exact hi sum and the lo sum
// form S13 to a few u^2 sigma, the product by s is a two_prod and the
// addition of c a two_sum, so q is correct to about an ulp of itself.
__device__ __forceinline__ double apply13_split(const Nb13& vh, const Nb13& vl, double c,
                                                double s) {
  const double sh = 20.0 * vh.c - 8.0 * ((vh.xm1 + vh.xp1) + (vh.ym1 + vh.yp1)) +
                    2.0 * ((vh.dmm + vh.dmp) + (vh.dpm + vh.dpp)) +
                    ((vh.xm2 + vh.xp2) + (vh.ym2 + vh.yp2));
  const double sl = 20.0 * vl.c - 8.0 * ((vl.xm1 + vl.xp1) + (vl.ym1 + vl.yp1)) +
                    2.0 * ((vl.dmm + vl.dmp) + (vl.dpm + vl.dpp)) +
                    ((vl.xm2 + vl.xp2) + (vl.ym2 + vl.yp2));
  double p, e1, w, e2;
  two_prod(s, sh, p, e1);
  e1 = fma(s, sl, e1);
  two_sum(c, p, w, e2);
  return w + (e1 + e2);
}

// ulp of a float64 value (0 for 0): spacing of the doubles around |v|.
__device__ __forceinline__ double ulp_of(double v) {
  int e;
  (void)frexp(v, &e);
  return v == 0.0 ? 0.0 : ldexp(1.0, e - 53);
}

}  // namespace bf
