// Device kernels of the biofilm-flow step: matrix-free 5- and 13-point
// operators, Chebyshev/Jacobi smoothing, cubic grid transfers, weighted
// reductions, Krylov vector updates and the pointwise step pieces.
//
// Operators (paper, Sec. 4 and Sec. 4.1):
//   L x   = n^2 (x[i-1] + x[i+1] + x[j-1] + x[j+1] - 4 x)   (matrix row 4,-1,-1,-1,-1
//           of Listing "Constructing the matrix with DMDA", scaled by -1/h^2)
//   A_CH x = x + s * (20 x - 8 axis + 2 diagonal + distance-two)  with s = c n^4,
//           the Cahn-Hilliard step operator I + c L^2 (Sec. 2.2, eq. modCH)
// Ghost rows by the two-layer reflection of eq. discreteBC, periodic x.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"
#include "stencil_ops.hpp"

namespace bf {

#define GRID_STRIDE(idx, total)                                                        \
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (total); \
       idx += (int64_t)gridDim.x * blockDim.x)

template <int OP, typename T>
__device__ __forceinline__ T stencil_at(const T* __restrict__ x, int i, int j, int n, int mask,
                                        T coef, T& center) {
  const Nb13T<T> v = gather<OP>(x, i, j, n, mask);
  center = v.c;
  return apply_vals<OP>(v, T(row_coef<OP>(double(coef), j, n)));
}

template <int OP>
__device__ __forceinline__ double residual_dd_at(const double* __restrict__ x, double bval, int i,
                                                 int j, int n, int mask, double coef) {
  return residual_dd_vals<OP>(gather<OP>(x, i, j, n, mask), bval, row_coef<OP>(coef, j, n));
}

// Batches on the one-thread-per-node kernels: blockIdx.y is the instance,
// fields are s0 (coarse fields of transfers: s1) elements apart, and coef
// (if set) holds each instance's coefficient record (see BatchCtx).
struct BArgs {
  int64_t s0, s1;
  const double* coef;
  int ia, ig, ia0;
};

static BArgs batch_args() {
  const BatchCtx& c = g_batch;
  BArgs B;
  B.s0 = c.count > 1 ? c.stride : 0;
  B.s1 = c.count > 1 ? c.stride_c : 0;
  B.coef = c.coef;
  B.ia = c.ia;
  B.ig = c.ig;
  B.ia0 = c.ia0;
  return B;
}
static int batch_count() { return g_batch.count > 1 ? g_batch.count : 1; }

__device__ __forceinline__ void inst_coef(const BArgs& B, OpDesc& A, double& a, double& g,
                                          double& a0) {
  if (B.coef) {
    const double* rc = B.coef + (int64_t)blockIdx.y * kCoefStride;
    A.coef = rc[0];
    A.dinv_int = rc[1];
    A.dinv_edge = rc[2];
    a = rc[3 + B.ia];
    g = rc[11 + B.ig];
    a0 = rc[3 + B.ia0];
  }
}

template <int OP, typename T = double>
__device__ __forceinline__ T dinv_at(const OpDesc& A, int j) {
  return T(row_dinv<OP>(A.dinv_int, A.dinv_edge, j, A.n));
}

// ------------------------------------------------------------------ operators
template <int OP>
__global__ void __launch_bounds__(kBlock) k_apply(OpDesc A, Geo G, const double* __restrict__ x,
                                                  double* __restrict__ y) {
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    double c;
    y[idx] = stencil_at<OP>(x, i, j, G.n, G.mask, A.coef, c);
  }
}

// ACC = 1 evaluates A p with the double-double stencil sum (q accurate to an
// ulp): the rounding of a plain float64 evaluation is amplified by c/h^4 and
// biased for smooth p, and it would accumulate in the recursive residual.
template <int OP, int ACC>
__global__ void __launch_bounds__(kBlock) k_apply_dot(OpDesc A, Geo G, const double* __restrict__ p,
                                                      double* __restrict__ q,
                                                      double* __restrict__ partials) {
  double acc = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    double c, v;
    if (ACC) {
      c = p[idx];
      v = -residual_dd_at<OP>(p, 0.0, i, j, G.n, G.mask, A.coef);
    } else {
      v = stencil_at<OP>(p, i, j, G.n, G.mask, A.coef, c);
    }
    q[idx] = v;
    acc += row_weight(j, G.n) * c * v;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <int OP, typename T>
__global__ void __launch_bounds__(kBlock) k_residual(OpDesc A, Geo G, const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ r,
                                                     double* __restrict__ partials, BArgs Bt) {
  double acc = 0.0;
  {
    double a_, g_, a0_;
    inst_coef(Bt, A, a_, g_, a0_);
    const int64_t o = (int64_t)blockIdx.y * Bt.s0;
    if (x) x += o;
    b += o;
    r += o;
  }
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    T v = b[idx];
    if (x) {
      T c;
      v -= stencil_at<OP>(x, i, j, G.n, G.mask, T(A.coef), c);
    }
    r[idx] = v;
    acc += row_weight(j, G.n) * double(v) * double(v);
  }
  if (partials) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// r = b - A x (double-double stencil sum).  partials[0..gridDim) receive
// ||r||_W^2 and partials[gridDim..2 gridDim) receive sum_W ulp(x)^2, from which
// the host forms the expected float64 representation floor of the residual:
// rounding x to float64 leaves errors uniform in +-ulp/2 (variance ulp^2/12),
// which A maps to a residual of norm^2 ~ sum_k ulp_k^2/12 * sum_j A_jk^2.
template <int OP>
__global__ void __launch_bounds__(kBlock) k_residual_dd(OpDesc A, Geo G,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ r,
                                                        double* __restrict__ partials) {
  double acc = 0.0, acc_ulp = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    const double v = residual_dd_at<OP>(x, b[idx], i, j, G.n, G.mask, A.coef);
    r[idx] = v;
    const double w = row_weight(j, G.n);
    acc += w * v * v;
    const double u = ulp_of(x[idx]);
    acc_ulp += w * u * u;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
  const double tu = block_sum(acc_ulp);
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = tu;
}

template <int OP, typename T>
__global__ void __launch_bounds__(kBlock) k_smooth(OpDesc A, Geo G, const T* __restrict__ x,
                                                   const T* xprev, const T* __restrict__ b,
                                                   T* xout, double a, double g, BArgs Bt) {
  {
    double a0_;
    inst_coef(Bt, A, a, g, a0_);
    const int64_t o = (int64_t)blockIdx.y * Bt.s0;
    x += o;
    if (xprev) xprev += o;
    b += o;
    xout += o;
  }
  const T ta = T(a), tg = T(g), coef = T(A.coef);
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    T c;
    const T ax = stencil_at<OP>(x, i, j, G.n, G.mask, coef, c);
    const T prev = xprev ? xprev[idx] : T(0);
    xout[idx] = c + ta * dinv_at<OP, T>(A, j) * (b[idx] - ax) + tg * (c - prev);
  }
}

template <int OP, typename T>
__global__ void __launch_bounds__(kBlock) k_smooth0(OpDesc A, Geo G, const T* __restrict__ b,
                                                    T* __restrict__ xout, double a, BArgs Bt) {
  {
    double g_, a0_;
    inst_coef(Bt, A, a, g_, a0_);
    if (Bt.coef) a = a0_;  // the first sweep takes a[ia0]
    const int64_t o = (int64_t)blockIdx.y * Bt.s0;
    b += o;
    xout += o;
  }
  const T ta = T(a);
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    xout[idx] = ta * dinv_at<OP, T>(A, j) * b[idx];
  }
}

template <int OP>
__global__ void __launch_bounds__(kBlock) k_jacobi_pc(OpDesc A, Geo G, const double* __restrict__ r,
                                                      double* __restrict__ z) {
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    z[idx] = dinv_at<OP>(A, j) * r[idx];
  }
}

// ------------------------------------------------------------------ transfers
// coarse = R fine and fine += P coarse (one thread per node; small levels).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(Geo F, Geo C, const T* __restrict__ fine,
                                                     T* __restrict__ coarse, BArgs Bt) {
  fine += (int64_t)blockIdx.y * Bt.s0;
  coarse += (int64_t)blockIdx.y * Bt.s1;
  GRID_STRIDE(idx, C.npts) {
    const int I = (int)(idx & C.mask), J = (int)(idx >> C.log2n);
    coarse[idx] = restrict_at(fine, F.n, F.mask, I, J);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_add(Geo F, Geo C, const T* __restrict__ coarse,
                                                        T* __restrict__ fine, BArgs Bt) {
  coarse += (int64_t)blockIdx.y * Bt.s1;
  fine += (int64_t)blockIdx.y * Bt.s0;
  GRID_STRIDE(idx, F.npts) {
    const int i = (int)(idx & F.mask), j = (int)(idx >> F.log2n);
    fine[idx] += prolong_at(coarse, C.n, C.mask, i, j);
  }
}

template <typename T>
__global__ void k_coarse_solve(int size, const double* __restrict__ G, const T* __restrict__ b,
                               T* __restrict__ x) {
  const int k = threadIdx.x;
  if (k < size) {
    double acc = 0.0;
    for (int l = 0; l < size; ++l) acc += G[k * size + l] * double(b[l]);
    x[k] = T(acc);
  }
}

// r32 = (float) r: the right-hand side of the float32 V-cycle.
__global__ void __launch_bounds__(kBlock) k_to_float(int64_t count, const double* __restrict__ x,
                                                     float* __restrict__ y) {
  GRID_STRIDE(idx, count) y[idx] = float(x[idx]);
}

__global__ void __launch_bounds__(kBlock) k_to_double(int64_t count, const float* __restrict__ x,
                                                      double* __restrict__ y) {
  GRID_STRIDE(idx, count) y[idx] = double(x[idx]);
}

// ------------------------------------------------------------------ reductions
__global__ void __launch_bounds__(kBlock) k_dot(Geo G, const double* __restrict__ x,
                                                const double* __restrict__ y,
                                                double* __restrict__ partials) {
  double acc = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    acc += row_weight(j, G.n) * x[idx] * (y ? y[idx] : 1.0);
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// partials of sum_W (x - y)
__global__ void __launch_bounds__(kBlock) k_wsum_diff(Geo G, const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      double* __restrict__ partials) {
  double acc = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    acc += row_weight(j, G.n) * (x[idx] - y[idx]);
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Sum of partials[0 .. nparts) by one workgroup of kFinTPB threads, each
// with four independent accumulators (the loads of a thread are issued
// together; a reducing kernel leaves up to 16384 partials, which one
// 256-thread workgroup summed in 12 us).  The order of the additions depends
// on nparts only, so the value is reproducible bit for bit.
constexpr int kFinTPB = 1024;

__device__ __forceinline__ double fin_sum(const double* __restrict__ p, int nparts) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int k = threadIdx.x;
  for (; k + 3 * kFinTPB < nparts; k += 4 * kFinTPB) {
    a0 += p[k];
    a1 += p[k + kFinTPB];
    a2 += p[k + 2 * kFinTPB];
    a3 += p[k + 3 * kFinTPB];
  }
  for (; k < nparts; k += kFinTPB) a0 += p[k];
  return block_sum_n<kFinTPB>((a0 + a1) + (a2 + a3));
}

// host (optional, F_STORE): pinned host memory that also receives the value
// and then, once the value is visible to the host, the sequence number hseq in
// host[S_HSEQ]: the host waits for that number instead of for an event or a
// copy (each system-scope fence writes the stores before it back to memory).
__global__ void __launch_bounds__(kFinTPB) k_finalize(const double* __restrict__ partials, int nparts,
                                                      double* __restrict__ scal, int mode, int slot,
                                                      double nn, double* __restrict__ host,
                                                      double hseq) {
  const double s = fin_sum(partials, nparts);
  if (threadIdx.x == 0) {
    switch (mode) {
      case F_STORE:
        scal[slot] = s;
        if (host) {
          host[slot] = s;
          __threadfence_system();
          host[S_HSEQ] = hseq;
          __threadfence_system();
        }
        break;
      case F_ALPHA:
        scal[S_PQ] = s;
        scal[S_ALPHA] = scal[S_RZ] / s;
        if (slot > 0) scal[slot] = scal[S_ALPHA];
        break;
      case F_BETA: {
        const double old = scal[S_RZ];
        scal[S_RZOLD] = old;
        scal[S_RZ] = s;
        scal[S_BETA] = s / old;
        break;
      }
      case F_MEAN:
        scal[S_MEAN] = s / nn;
        break;
    }
  }
}

__global__ void __launch_bounds__(64) k_residual_norms(const double* __restrict__ scal, double csq,
                                                     double* __restrict__ out) {
  if (threadIdx.x == 0) {
    const double bn = sqrt(scal[S_BN2]);
    const double d = bn > 0.0 ? bn : 1.0;
    out[0] = sqrt(scal[S_RTRUE]) / d;
    out[1] = sqrt(scal[S_ULP2] / 12.0 * csq) / d;
    out[2] = bn;
  }
}

// Flexible (Polak-Ribiere) CG coefficient from two groups of partials:
// rho = sum partials[0..np) = <r_k, z_k>_W, gamma = sum partials[np..2 np) =
// <z_k, q_{k-1}>_W; beta = (rho - <z_k, r_{k-1}>) / rho_old = -alpha gamma / rho_old
// since r_k = r_{k-1} - alpha q_{k-1}.
__global__ void __launch_bounds__(kFinTPB) k_finalize_flex(const double* __restrict__ partials,
                                                           int nparts, double* __restrict__ scal) {
  const double rho = fin_sum(partials, nparts);
  const double gamma = fin_sum(partials + nparts, nparts);
  if (threadIdx.x == 0) {
    const double old = scal[S_RZ];
    scal[S_RZOLD] = old;
    scal[S_RZ] = rho;
    scal[S_BETA] = -scal[S_ALPHA] * gamma / old;
  }
}

// Naive form of the fused CG step (small levels; see stream_cg_p).
template <int OP>
__global__ void __launch_bounds__(kBlock) k_cg_p(OpDesc A, Geo G, const double* __restrict__ z,
                                                 const double* __restrict__ p_old,
                                                 double* __restrict__ p_new,
                                                 double* __restrict__ q, double* __restrict__ x,
                                                 const double* __restrict__ scal, int first,
                                                 double* __restrict__ partials) {
  const double beta = first ? 0.0 : scal[S_BETA];
  const double alpha = first ? 0.0 : scal[S_ALPHA];
  double acc = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    Nb13 v = gather<OP>(z, i, j, G.n, G.mask);
    if (!first) {
      const Nb13 w = gather<OP>(p_old, i, j, G.n, G.mask);
      v.c += beta * w.c;
      v.xm1 += beta * w.xm1;
      v.xp1 += beta * w.xp1;
      v.ym1 += beta * w.ym1;
      v.yp1 += beta * w.yp1;
      if (OP == 1) {
        v.dmm += beta * w.dmm;
        v.dmp += beta * w.dmp;
        v.dpm += beta * w.dpm;
        v.dpp += beta * w.dpp;
        v.xm2 += beta * w.xm2;
        v.xp2 += beta * w.xp2;
        v.ym2 += beta * w.ym2;
        v.yp2 += beta * w.yp2;
      }
      x[idx] += alpha * w.c;
    }
    const double cj = row_coef<OP>(A.coef, j, G.n);
    const double qv = OP == 1 ? -residual_dd_vals<OP>(v, 0.0, cj) : apply_vals<OP>(v, cj);
    q[idx] = qv;
    p_new[idx] = v.c;
    acc += row_weight(j, G.n) * v.c * qv;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_r_update(Geo G, double* __restrict__ r,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ scal,
                                                     double* __restrict__ partials,
                                                     float* __restrict__ r32) {
  const double alpha = scal[S_ALPHA];
  double acc = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    const double rv = r[idx] - alpha * q[idx];
    r[idx] = rv;
    if (r32) r32[idx] = float(rv);
    acc += row_weight(j, G.n) * rv * rv;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename PT>
__global__ void __launch_bounds__(kBlock) k_x_update(Geo G, double* __restrict__ x,
                                                     const PT* __restrict__ p,
                                                     const double* __restrict__ scal) {
  const double alpha = scal[S_ALPHA];
  GRID_STRIDE(idx, G.npts) x[idx] += alpha * double(p[idx]);
}

// x += sum_i alpha_i p_i over m float32 search directions (alpha_i =
// alpha[i]): the iterate update of up to kRing CG steps in one pass.  Four
// nodes per thread (npts is a multiple of 4); the sum is formed in float64
// registers in the order of i and added to x once.
struct RingPtrs {
  const float* p[kRing];
};

typedef float bf_f4 __attribute__((ext_vector_type(4)));
typedef double bf_d2 __attribute__((ext_vector_type(2)));

template <int M>
__global__ void __launch_bounds__(kBlock) k_x_accum(int64_t nquad, double* __restrict__ x,
                                                   RingPtrs R, const double* __restrict__ alpha) {
  double a[M];
#pragma unroll
  for (int i = 0; i < M; ++i) a[i] = alpha[i];
  GRID_STRIDE(t, nquad) {
    // every value is used once: non-temporal loads and stores
    bf_f4 pv[M];
#pragma unroll
    for (int i = 0; i < M; ++i)
      pv[i] = __builtin_nontemporal_load(reinterpret_cast<const bf_f4*>(R.p[i]) + t);
    bf_d2* xq = reinterpret_cast<bf_d2*>(x) + 2 * t;
    bf_d2 x0 = __builtin_nontemporal_load(xq), x1 = __builtin_nontemporal_load(xq + 1);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      s0 += a[i] * double(pv[i].x);
      s1 += a[i] * double(pv[i].y);
      s2 += a[i] * double(pv[i].z);
      s3 += a[i] * double(pv[i].w);
    }
    x0.x += s0;
    x0.y += s1;
    x1.x += s2;
    x1.y += s3;
    __builtin_nontemporal_store(x0, xq);
    __builtin_nontemporal_store(x1, xq + 1);
  }
}

// The start of a solve from a zero iterate with a projected right-hand side:
// y = x - m (m = scal[S_MEAN]) into b and into the residual r (r = b - A 0),
// (float) y into r32 when given, and partials of ||y||_W^2.
__global__ void __launch_bounds__(kBlock) k_project_start(Geo G, const double* __restrict__ x,
                                                          double* __restrict__ b,
                                                          double* __restrict__ r,
                                                          float* __restrict__ r32,
                                                          const double* __restrict__ scal,
                                                          double* __restrict__ partials) {
  const double m = scal[S_MEAN];
  double acc = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    const double y = x[idx] - m;
    b[idx] = y;
    r[idx] = y;
    if (r32) r32[idx] = float(y);
    acc += row_weight(j, G.n) * y * y;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_sub_mean(Geo G, const double* x, double* y,
                                                     const double* __restrict__ scal,
                                                     double sign) {
  const double m = sign * scal[S_MEAN];
  GRID_STRIDE(idx, G.npts) y[idx] = x[idx] - m;
}

__global__ void __launch_bounds__(kBlock) k_fill(int64_t count, double* __restrict__ x, double v) {
  GRID_STRIDE(idx, count) x[idx] = v;
}

__global__ void __launch_bounds__(kBlock) k_copy(int64_t count, const double* __restrict__ x,
                                                 double* __restrict__ y) {
  GRID_STRIDE(idx, count) y[idx] = x[idx];
}

// y = x with 16-byte accesses per lane (count even, 16-byte aligned): the
// access pattern of the streaming stencil kernels, used as a calibration
// kernel of known traffic.
__global__ void __launch_bounds__(kBlock) k_copy2(int64_t pairs, const double2* __restrict__ x,
                                                  double2* __restrict__ y) {
  GRID_STRIDE(idx, pairs) y[idx] = x[idx];
}

__global__ void k_fill_i32(int count, int32_t* x, int32_t v) {
  GRID_STRIDE(idx, count) x[idx] = v;
}

// ------------------------------------------------------------------ step pieces
__device__ __forceinline__ double mu_fh(double f, double inv_npoly, double chi) {
  return log(f) * inv_npoly + inv_npoly - log(1.0 - f) - 1.0 + chi * (1.0 - 2.0 * f);
}

__device__ __forceinline__ double clampd(double f, double lo, double hi) {
  return fmin(fmax(f, lo), hi);
}

// Flory-Huggins right-hand side (Sec. 2.2, eq. modCH with the parameters chi,
// N of the Sec. 5 table): b = base + dtM n^2 (axis - 4 c) of mu, mu =
// mu_FH(clamp(phi*)) with phi* = phi, or the extrapolation 3/2 phi - 1/2 prev
// when prev is given (Crank-Nicolson); clamped nodes are counted; base may
// alias b.
//
// One pass (k_ch_rhs_tile, grids of n >= 128): a workgroup owns a tile of
// kRhsRows x kRhsCols nodes, evaluates mu once per node of the tile widened
// by the Laplacian's reach (one row above and below, one column either side)
// into LDS, and applies the 5-point Laplacian from there, so phi is read from
// HBM once, mu never leaves the chip, and the logarithms -- the bulk of the
// work: two float64 logs per node -- are evaluated (18 x 130) / (16 x 128) =
// 1.14 times per node.  Smaller grids take two passes (k_mu, k_lap_axpy).
constexpr int kRhsCols = 128;  // 64 lane pairs
constexpr int kRhsRows = 16;

__global__ void __launch_bounds__(kBlock) k_ch_rhs_tile(Geo G, int64_t stride, int strips,
                                                        const double* __restrict__ phi,
                                                        const double* __restrict__ prev,
                                                        const double* base, double* b,
                                                        RhsCoef C0,
                                                        const double* __restrict__ icoef,
                                                        int icoef_stride,
                                                        int32_t* __restrict__ clamp_count) {
  __shared__ double mu[kRhsRows + 2][kRhsCols + 2];
  __shared__ int cnt_s;
  const int inst = blockIdx.y;
  RhsCoef C = C0;
  if (icoef) {
    const double* rc = icoef + (int64_t)inst * icoef_stride;
    C.dtMn2 = rc[0];
    C.inv_npoly = rc[1];
    C.chi = rc[2];
    C.lo = rc[3];
    C.hi = rc[4];
  }
  const int64_t off = (int64_t)inst * stride;
  phi += off;
  if (prev) prev += off;
  base += off;
  b += off;
  const int n = G.n, mask = G.mask;
  const int rg = blockIdx.x / strips;
  const int c0 = (blockIdx.x - rg * strips) * kRhsCols;
  const int j0 = rg * kRhsRows;
  const int rows = min(j0 + kRhsRows, n + 1) - j0;  // output rows of the tile
  if (threadIdx.x == 0) cnt_s = 0;
  int cnt = 0;
  // mu on rows j0-1 .. j0+rows (reflected), columns c0 .. c0+127 (two per thread)
  for (int s = threadIdx.x; s < (rows + 2) * 64; s += kBlock) {
    const int r = s >> 6, l = s & 63;
    const int64_t idx = (int64_t)refl(j0 - 1 + r, n) * n + c0 + 2 * l;
    const double2 pv = *reinterpret_cast<const double2*>(phi + idx);
    double f0 = pv.x, f1 = pv.y;
    if (prev) {
      const double2 qv = *reinterpret_cast<const double2*>(prev + idx);
      f0 = 1.5 * f0 - 0.5 * qv.x;
      f1 = 1.5 * f1 - 0.5 * qv.y;
    }
    if (r >= 1 && r <= rows)
      cnt += ((f0 < C.lo || f0 > C.hi) ? 1 : 0) + ((f1 < C.lo || f1 > C.hi) ? 1 : 0);
    mu[r][1 + 2 * l] = mu_fh(clampd(f0, C.lo, C.hi), C.inv_npoly, C.chi);
    mu[r][2 + 2 * l] = mu_fh(clampd(f1, C.lo, C.hi), C.inv_npoly, C.chi);
  }
  // the columns c0 - 1 and c0 + 128 (wrapped)
  for (int s = threadIdx.x; s < (rows + 2) * 2; s += kBlock) {
    const int r = s >> 1, side = s & 1;
    const int col = side ? ((c0 + kRhsCols) & mask) : ((c0 - 1) & mask);
    const int64_t idx = (int64_t)refl(j0 - 1 + r, n) * n + col;
    const double f = prev ? 1.5 * phi[idx] - 0.5 * prev[idx] : phi[idx];
    mu[r][side ? kRhsCols + 1 : 0] = mu_fh(clampd(f, C.lo, C.hi), C.inv_npoly, C.chi);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < rows * 64; s += kBlock) {
    const int r = s >> 6, l = s & 63;
    const int64_t idx = (int64_t)(j0 + r) * n + c0 + 2 * l;
    const double* m = &mu[r + 1][1 + 2 * l];
    const double* mu_dn = &mu[r][1 + 2 * l];
    const double* mu_up = &mu[r + 2][1 + 2 * l];
    const double lap0 = (m[-1] + m[1]) + (mu_dn[0] + mu_up[0]) - 4.0 * m[0];
    const double lap1 = (m[0] + m[2]) + (mu_dn[1] + mu_up[1]) - 4.0 * m[1];
    const double2 bv = *reinterpret_cast<const double2*>(base + idx);
    double2 out;
    out.x = bv.x + C.dtMn2 * lap0;
    out.y = bv.y + C.dtMn2 * lap1;
    *reinterpret_cast<double2*>(b + idx) = out;
  }
  if (clamp_count) {
    if (cnt) atomicAdd(&cnt_s, cnt);
    __syncthreads();
    if (threadIdx.x == 0 && cnt_s) atomicAdd(clamp_count + inst, cnt_s);
  }
}

// Two-pass form (grids below 128 columns): mu once per node, then the
// Laplacian.
__global__ void __launch_bounds__(kBlock) k_mu(Geo G, const double* __restrict__ phi,
                                               const double* __restrict__ prev,
                                               double* __restrict__ mu, double inv_npoly,
                                               double chi, double lo, double hi,
                                               int32_t* clamp_count) {
  int cnt = 0;
  GRID_STRIDE(idx, G.npts) {
    const double c = prev ? 1.5 * phi[idx] - 0.5 * prev[idx] : phi[idx];
    cnt += (c < lo || c > hi) ? 1 : 0;
    mu[idx] = mu_fh(clampd(c, lo, hi), inv_npoly, chi);
  }
  if (clamp_count && cnt) atomicAdd(clamp_count, cnt);
}

__global__ void __launch_bounds__(kBlock) k_lap_axpy(Geo G, const double* __restrict__ mu,
                                                     const double* base, double* b,
                                                     double scale) {
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    const int n = G.n;
    const double* r0 = mu + (int64_t)j * n;
    const double lap = (r0[(i - 1) & G.mask] + r0[(i + 1) & G.mask]) +
                       (mu[(int64_t)refl(j - 1, n) * n + i] + mu[(int64_t)refl(j + 1, n) * n + i]) -
                       4.0 * r0[i];
    b[idx] = base[idx] + scale * lap;
  }
}

// ------------------------------------------------------------------ variable mobility
// A_m x = x + c L_m L x with L_m f = n^2 sum_faces m_face (f_nb - f),
// m_face = (m + m_nb)/2 (the phi-dependent mobility of the modified
// Cahn-Hilliard equation), ghost rows reflected for x and m alike.  The whole
// evaluation is carried in double-double (L x at the five points as exact
// Sum2 sums, the face fluxes, the scaling by c, the addition of x, and for
// MODE 1 the subtraction from b), so the result is accurate to a few ulps of
// itself although c n^4 m reaches 1e7.  One node per thread: the 13 values
// of x and 5 of m around a node come from cache.
//   MODE 0: y = A_m x.
//   MODE 1: y = b - A_m x, partials of ||y||_W^2 and of
//           sum_W ulp(x_k)^2 * colsq_k, colsq_k = (1 + 20 t)^2 + 276 t^2 with
//           t = c n^4 m_k: the squared column norm of the constant-mobility
//           operator at the local mobility, so that the representation floor
//           follows the mobility field (it varies by an order of magnitude).
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_mob(Geo G, double c, const double* __restrict__ m,
                                                const double* __restrict__ x,
                                                const double* __restrict__ b,
                                                double* __restrict__ y,
                                                double* __restrict__ partials) {
#pragma clang fp contract(off)
  const int n = G.n, mask = G.mask;
  const double n2 = (double)n * n;
  double acc = 0.0, acc_ulp = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & mask), j = (int)(idx >> G.log2n);
    auto X = [&](int jj, int ii) { return x[(int64_t)refl(jj, n) * n + (ii & mask)]; };
    auto T = [&](int jj, int ii) {  // (L x) at (ii, jj) in double-double
      const DD s = dd_lap_sum(X(jj, ii - 1), X(jj, ii + 1), X(jj - 1, ii), X(jj + 1, ii),
                              X(jj, ii));
      return DD{s.hi * n2, s.lo * n2};
    };
    const double mc = m[idx];
    const DD tc = T(j, i);
    const int dj[4] = {0, 0, -1, 1}, di[4] = {-1, 1, 0, 0};
    DD f{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int jj = j + dj[k], ii = i + di[k];
      const double mf = 0.5 * (mc + m[(int64_t)refl(jj, n) * n + (ii & mask)]);
      f = dd_add(f, dd_mul_d(dd_sub(T(jj, ii), tc), mf));
    }
    f = DD{f.hi * n2, f.lo * n2};
    const double xc = x[idx];
    const DD ax = dd_add_d(dd_mul_d(f, c), xc);
    if (MODE == 0) {
      y[idx] = ax.hi + ax.lo;
    } else {
      const DD r = dd_add_d(DD{-ax.hi, -ax.lo}, b[idx]);
      const double rv = r.hi + r.lo;
      y[idx] = rv;
      const double w = row_weight(j, n);
      acc += w * rv * rv;
      const double u = ulp_of(xc);
      const double t = c * n2 * n2 * mc;
      acc_ulp += w * u * u * ((1.0 + 20.0 * t) * (1.0 + 20.0 * t) + 276.0 * t * t);
    }
  }
  if (MODE == 1) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
    const double tu = block_sum(acc_ulp);
    if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = tu;
  }
}

// Variable-mobility multigrid (the preconditioner of bf_solve_ch_mob on the
// levels above the coarse tail): the operator rediscretised on each level
// with that level's node mobilities, applied in plain T arithmetic (a
// preconditioner needs no more), one node per thread.  cs = c n^4 of the
// level; the smoother's diagonal is the interior one, 1 + 5 cs sum_faces m_f.
template <typename T>
__device__ __forceinline__ T mob_apply_at(const T* __restrict__ x, const T* __restrict__ m, int i,
                                          int j, int n, int mask, T cs, T& diag) {
  auto X = [&](int jj, int ii) { return x[(int64_t)refl(jj, n) * n + (ii & mask)]; };
  auto Lh = [&](int jj, int ii) {
    return (X(jj, ii - 1) + X(jj, ii + 1)) + (X(jj - 1, ii) + X(jj + 1, ii)) - T(4) * X(jj, ii);
  };
  const T mc = m[(int64_t)j * n + i];
  const T tc = Lh(j, i);
  const int dj[4] = {0, 0, -1, 1}, di[4] = {-1, 1, 0, 0};
  T f = T(0), sm = T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int jj = j + dj[k], ii = i + di[k];
    const T mf = T(0.5) * (mc + m[(int64_t)refl(jj, n) * n + (ii & mask)]);
    f += mf * (Lh(jj, ii) - tc);
    sm += mf;
  }
  diag = T(1) + T(5) * cs * sm;
  return X(j, i) + cs * f;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_mob_smooth(Geo G, T cs, const T* __restrict__ m,
                                                       const T* __restrict__ x, const T* xprev,
                                                       const T* __restrict__ b, T* xout, T a,
                                                       T g) {
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    T d;
    const T ax = mob_apply_at(x, m, i, j, G.n, G.mask, cs, d);
    const T c = x[idx];
    const T prev = xprev ? xprev[idx] : T(0);
    xout[idx] = c + a / d * (b[idx] - ax) + g * (c - prev);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_mob_smooth0(Geo G, T cs, const T* __restrict__ m,
                                                        const T* __restrict__ b,
                                                        T* __restrict__ xout, T a0) {
  const int n = G.n;
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    const T mc = m[idx];
    T sm = T(0);
    const int dj[4] = {0, 0, -1, 1}, di[4] = {-1, 1, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      sm += T(0.5) * (mc + m[(int64_t)refl(j + dj[k], n) * n + ((i + di[k]) & G.mask)]);
    xout[idx] = a0 / (T(1) + T(5) * cs * sm) * b[idx];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_mob_residual(Geo G, T cs, const T* __restrict__ m,
                                                         const T* __restrict__ x,
                                                         const T* __restrict__ b,
                                                         T* __restrict__ r) {
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    T d;
    r[idx] = b[idx] - mob_apply_at(x, m, i, j, G.n, G.mask, cs, d);
  }
}

// coarse m = fine m at the coinciding (even) nodes
template <typename T>
__global__ void __launch_bounds__(kBlock) k_inject(Geo F, Geo C, const T* __restrict__ fine,
                                                   T* __restrict__ coarse) {
  GRID_STRIDE(idx, C.npts) {
    const int I = (int)(idx & C.mask), J = (int)(idx >> C.log2n);
    coarse[idx] = fine[(int64_t)(2 * J) * F.n + 2 * I];
  }
}

// Variable-mobility right-hand side: m = M clamp(phi) (written), then
// b = phi + dt L_m mu with mu from k_mu (plain float64).
__global__ void __launch_bounds__(kBlock) k_mob_field(Geo G, const double* __restrict__ phi,
                                                      double* __restrict__ m, double M, double lo,
                                                      double hi) {
  GRID_STRIDE(idx, G.npts) m[idx] = M * clampd(phi[idx], lo, hi);
}

__global__ void __launch_bounds__(kBlock) k_mob_rhs(Geo G, const double* __restrict__ phi,
                                                    const double* __restrict__ mu,
                                                    const double* __restrict__ m,
                                                    double* __restrict__ b, double scale) {
  const int n = G.n, mask = G.mask;
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & mask), j = (int)(idx >> G.log2n);
    const double mc = m[idx], uc = mu[idx];
    const int dj[4] = {0, 0, -1, 1}, di[4] = {-1, 1, 0, 0};
    double f = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t o = (int64_t)refl(j + dj[k], n) * n + ((i + di[k]) & mask);
      f += 0.5 * (mc + m[o]) * (mu[o] - uc);
    }
    b[idx] = phi[idx] + scale * f;
  }
}

// rhs = (u[i+1] - u[i-1] + v[j+1] - v[j-1]) * scale, v odd across the walls.
__global__ void __launch_bounds__(kBlock) k_divergence(Geo G, const double* __restrict__ u,
                                                       const double* __restrict__ v,
                                                       double* __restrict__ rhs, double scale) {
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    const int n = G.n;
    const double* ur = u + (int64_t)j * n;
    const double vp = (j == n) ? -v[(int64_t)(n - 1) * n + i] : v[idx + n];
    const double vm = (j == 0) ? -v[(int64_t)n + i] : v[idx - n];
    rhs[idx] = ((ur[(i + 1) & G.mask] - ur[(i - 1) & G.mask]) + (vp - vm)) * scale;
  }
}

__global__ void __launch_bounds__(kBlock) k_velocity(Geo G, const double* __restrict__ p,
                                                     const double* us, const double* vs,
                                                     double* u, double* v, double scale) {
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    const int n = G.n;
    const double* pr = p + (int64_t)j * n;
    const double gx = pr[(i + 1) & G.mask] - pr[(i - 1) & G.mask];
    const double gy = p[(int64_t)refl(j + 1, n) * n + i] - p[(int64_t)refl(j - 1, n) * n + i];
    if (u) u[idx] = us[idx] - scale * gx;
    if (v) v[idx] = vs[idx] - scale * gy;
  }
}

// Right-hand sides of the momentum predictor (one node per thread): on the
// interior rows f - dt (u f_x + v f_y) + e L_D f for f = u and f = v (central
// differences; the y differences and the Laplacian read the wall rows as
// they are); on the wall rows the Dirichlet data (bu: 0 at the bottom, U at
// the top; bv: 0).  h1 = n/2 = 1/(2h), h2 = n^2 = 1/h^2.
__global__ void __launch_bounds__(kBlock) k_momentum_rhs(Geo G, const double* __restrict__ u,
                                                         const double* __restrict__ v, double dt,
                                                         double e, double U,
                                                         double* __restrict__ bu,
                                                         double* __restrict__ bv) {
  const int n = G.n;
  const double h1 = 0.5 * n, h2 = (double)n * n;
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    if (j == 0 || j == n) {
      bu[idx] = j == 0 ? 0.0 : U;
      bv[idx] = 0.0;
      continue;
    }
    const int64_t im = (int64_t)j * n + ((i - 1) & G.mask), ip = (int64_t)j * n + ((i + 1) & G.mask);
    const int64_t jm = idx - n, jp = idx + n;
    const double uc = u[idx], vc = v[idx];
    const double ux = (u[ip] - u[im]) * h1, uy = (u[jp] - u[jm]) * h1;
    const double vx = (v[ip] - v[im]) * h1, vy = (v[jp] - v[jm]) * h1;
    const double lu = (u[im] + u[ip] + u[jm] + u[jp] - 4.0 * uc) * h2;
    const double lv = (v[im] + v[ip] + v[jm] + v[jp] - 4.0 * vc) * h2;
    bu[idx] = uc - dt * (uc * ux + vc * uy) + e * lu;
    bv[idx] = vc - dt * (uc * vx + vc * vy) + e * lv;
  }
}

// ------------------------------------------------------------------ advection, adjoint
// D(phi; u, v)_ij * 2h = (phi u)_{i+1} - (phi u)_{i-1} + (phi v)_{j+1} - (phi v)_{j-1}
// with phi even and v odd across the walls (phi v odd): wall rows fold the
// ghost onto the first interior row.
__device__ __forceinline__ double flux_div2h(const double* phi, const double* u, const double* v,
                                             int i, int j, int n, int mask) {
  const double* pr = phi + (int64_t)j * n;
  const double* ur = u + (int64_t)j * n;
  const int im = (i - 1) & mask, ip = (i + 1) & mask;
  const double dx = pr[ip] * ur[ip] - pr[im] * ur[im];
  double dy;
  if (j == 0) {
    dy = 2.0 * phi[(int64_t)n + i] * v[(int64_t)n + i];
  } else if (j == n) {
    const int64_t o = (int64_t)(n - 1) * n + i;
    dy = -2.0 * phi[o] * v[o];
  } else {
    const int64_t op = (int64_t)(j + 1) * n + i, om = (int64_t)(j - 1) * n + i;
    dy = phi[op] * v[op] - phi[om] * v[om];
  }
  return dx + dy;
}

// b -= dt D(phi; u, v)   (scale = dt / (2h))
__global__ void __launch_bounds__(kBlock) k_advect_sub(Geo G, const double* __restrict__ phi,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ v,
                                                       double* __restrict__ b, double scale) {
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    b[idx] -= scale * flux_div2h(phi, u, v, i, j, G.n, G.mask);
  }
}

// y = x * w_j (inverse = 0) or x / w_j (inverse = 1), w = trapezoid row weights.
__global__ void __launch_bounds__(kBlock) k_wscale(Geo G, const double* __restrict__ x,
                                                   double* __restrict__ y, int inverse) {
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    const double w = row_weight(j, G.n);
    y[idx] = inverse ? x[idx] / w : x[idx] * w;
  }
}

// Adjoint right-hand side of one step, from e = W^{-1} eta (the solution of
// A e = W^{-1} lam_next, so eta = W e = A^{-T} lam_next):
//   lam = eta + dtM mu'(phi) (L^T eta) - dt D^T eta,  L^T eta = W L e,
//   partials[b]          of sum (L^T eta)(1 - 2 clamp(phi))   (dJ/dchi / dtM)
//   partials[nparts + b] of sum eta D(phi; du, dv)             (dJ/dU / -dt)
// D^T eta = u (eta_{i-1} - eta_{i+1})/(2h) + v (em - ep) with
//   em = eta_{j-1}/(2h) for j >= 2, eta_0/h for j = 1, 0 for j = 0;
//   ep = eta_{j+1}/(2h) for j <= n-2, eta_n/h for j = n-1, 0 for j = n.
__global__ void __launch_bounds__(kBlock) k_adjoint_rhs(Geo G, const double* __restrict__ e,
                                                        const double* __restrict__ phi,
                                                        const double* __restrict__ u,
                                                        const double* __restrict__ v,
                                                        const double* __restrict__ du,
                                                        const double* __restrict__ dv,
                                                        double* __restrict__ lam, AdjCoef C,
                                                        double* __restrict__ partials) {
  double a1 = 0.0, a2 = 0.0;
  const int n = G.n;
  const double n2 = (double)n * (double)n, inv2h = 0.5 * (double)n;
  GRID_STRIDE(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    const double wj = row_weight(j, n);
    const double* er = e + (int64_t)j * n;
    const int im = (i - 1) & G.mask, ip = (i + 1) & G.mask;
    const double ec = er[i];
    const double le = n2 * ((er[im] + er[ip]) + (e[(int64_t)refl(j - 1, n) * n + i] +
                                                 e[(int64_t)refl(j + 1, n) * n + i]) -
                            4.0 * ec);
    const double lt = wj * le;
    const double eta = wj * ec;
    const double p = phi[idx];
    const bool active = p >= C.lo && p <= C.hi;
    const double ph = p < C.lo ? C.lo : (p > C.hi ? C.hi : p);
    const double mup = active ? (C.inv_npoly / ph + 1.0 / (1.0 - ph) - 2.0 * C.chi) : 0.0;
    double out = eta + C.dtM * mup * lt;
    if (u) {
      const double dxt = u[idx] * wj * (er[im] - er[ip]) * inv2h;
      double em = 0.0, epp = 0.0;
      if (j >= 2) em = row_weight(j - 1, n) * e[idx - n] * inv2h;
      else if (j == 1) em = row_weight(0, n) * e[i] * 2.0 * inv2h;
      if (j <= n - 2) epp = row_weight(j + 1, n) * e[idx + n] * inv2h;
      else if (j == n - 1) epp = row_weight(n, n) * e[(int64_t)n * n + i] * 2.0 * inv2h;
      out -= C.dt * (dxt + v[idx] * (em - epp));
    }
    lam[idx] = out;
    a1 += lt * (1.0 - 2.0 * ph);
    if (du) a2 += eta * flux_div2h(phi, du, dv, i, j, n, G.mask) * inv2h;
  }
  const double s1 = block_sum(a1);
  const double s2 = block_sum(a2);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s1;
    partials[gridDim.x + blockIdx.x] = s2;
  }
}

// ------------------------------------------------------------------ GMRES pieces
constexpr int kMdotGroup = 8;

__global__ void __launch_bounds__(kBlock) k_mdot(Geo G, const double* __restrict__ V, int m, int k0,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ partials) {
  double acc[kMdotGroup];
#pragma unroll
  for (int k = 0; k < kMdotGroup; ++k) acc[k] = 0.0;
  const int kn = min(kMdotGroup, m - k0);
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    const double ww = row_weight(j, G.n) * w[idx];
#pragma unroll
    for (int k = 0; k < kMdotGroup; ++k)
      if (k < kn) acc[k] += V[(int64_t)(k0 + k) * G.npts + idx] * ww;
  }
  for (int k = 0; k < kn; ++k) {
    const double t = block_sum(acc[k]);
    if (threadIdx.x == 0) partials[(int64_t)(k0 + k) * gridDim.x + blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock) k_finalize_multi(const double* __restrict__ partials,
                                                           int nparts, double* __restrict__ scal,
                                                           int slot) {
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int t = threadIdx.x; t < nparts; t += kBlock) acc += partials[(int64_t)k * nparts + t];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) scal[slot + k] = s;
}

__global__ void __launch_bounds__(kBlock) k_maxpy(Geo G, const double* __restrict__ V, int m,
                                                  const double* __restrict__ h,
                                                  double* __restrict__ w,
                                                  double* __restrict__ partials) {
  double acc = 0.0;
  GRID_STRIDE(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    double v = w[idx];
    for (int k = 0; k < m; ++k) v -= h[k] * V[(int64_t)k * G.npts + idx];
    w[idx] = v;
    acc += row_weight(j, G.n) * v * v;
  }
  if (partials) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock) k_axpy_multi(Geo G, const double* __restrict__ Z, int m,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ x) {
  GRID_STRIDE(idx, G.npts) {
    double v = x[idx];
    for (int k = 0; k < m; ++k) v += y[k] * Z[(int64_t)k * G.npts + idx];
    x[idx] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_scale(Geo G, const double* __restrict__ x,
                                                  double* __restrict__ y,
                                                  const double* __restrict__ scal, int slot,
                                                  int invert_sqrt) {
  const double s = invert_sqrt ? 1.0 / sqrt(scal[slot]) : scal[slot];
  GRID_STRIDE(idx, G.npts) y[idx] = s * x[idx];
}

// ------------------------------------------------------------------ launchers
#define LAUNCH(kern, blocks, st, ...) hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, st, __VA_ARGS__)
// Launch over the instances of the current batch (grid.y = instance).
#define LAUNCH_B(kern, blocks, st, ...) \
  hipLaunchKernelGGL(kern, dim3(blocks, batch_count()), dim3(kBlock), 0, st, __VA_ARGS__)

void launch_apply(const OpDesc& A, const double* x, double* y, hipStream_t st) {
  if (stream_ok(A.n)) {
    stream_apply(A, x, y, st);
    return;
  }
  const Geo G = make_geo(A.n);
  if (A.op == 0)
    LAUNCH(k_apply<0>, ew_blocks(G.npts), st, A, G, x, y);
  else if (A.op == 2)
    LAUNCH(k_apply<2>, ew_blocks(G.npts), st, A, G, x, y);
  else
    LAUNCH(k_apply<1>, ew_blocks(G.npts), st, A, G, x, y);
}

int launch_apply_dot(const OpDesc& A, const double* p, double* q, double* partials, int nparts,
                     hipStream_t st, bool accurate) {
  if (stream_ok(A.n)) return stream_apply_dot(A, p, q, partials, accurate, st);
  const Geo G = make_geo(A.n);
  if (A.op == 0) {
    if (accurate)
      LAUNCH((k_apply_dot<0, 1>), nparts, st, A, G, p, q, partials);
    else
      LAUNCH((k_apply_dot<0, 0>), nparts, st, A, G, p, q, partials);
  } else if (A.op == 2) {
    if (accurate)
      LAUNCH((k_apply_dot<2, 1>), nparts, st, A, G, p, q, partials);
    else
      LAUNCH((k_apply_dot<2, 0>), nparts, st, A, G, p, q, partials);
  } else {
    if (accurate)
      LAUNCH((k_apply_dot<1, 1>), nparts, st, A, G, p, q, partials);
    else
      LAUNCH((k_apply_dot<1, 0>), nparts, st, A, G, p, q, partials);
  }
  return nparts;
}

template <typename T>
int launch_residual(const OpDesc& A, const T* x, const T* b, T* r, double* partials, int nparts,
                    hipStream_t st) {
  if (x && stream_ok(A.n, sizeof(T))) return stream_residual<T>(A, x, b, r, partials, st);
  const Geo G = make_geo(A.n);
  const int blocks = partials ? nparts : ew_blocks(G.npts);
  if (A.op == 0)
    LAUNCH_B((k_residual<0, T>), blocks, st, A, G, x, b, r, partials, batch_args());
  else if (A.op == 2)
    LAUNCH_B((k_residual<2, T>), blocks, st, A, G, x, b, r, partials, batch_args());
  else
    LAUNCH_B((k_residual<1, T>), blocks, st, A, G, x, b, r, partials, batch_args());
  return blocks * batch_count();
}
template int launch_residual<double>(const OpDesc&, const double*, const double*, double*,
                                     double*, int, hipStream_t);
template int launch_residual<float>(const OpDesc&, const float*, const float*, float*, double*,
                                    int, hipStream_t);

int launch_residual_dd(const OpDesc& A, const double* x, const double* b, double* r,
                       double* partials, int nparts, hipStream_t st) {
  if (stream_ok(A.n)) return stream_residual_dd(A, x, b, r, partials, st);
  const Geo G = make_geo(A.n);
  if (A.op == 0)
    LAUNCH(k_residual_dd<0>, nparts, st, A, G, x, b, r, partials);
  else if (A.op == 2)
    LAUNCH(k_residual_dd<2>, nparts, st, A, G, x, b, r, partials);
  else
    LAUNCH(k_residual_dd<1>, nparts, st, A, G, x, b, r, partials);
  return nparts;
}

template <typename T>
void launch_smooth(const OpDesc& A, const T* x, const T* xprev, const T* b, T* xout, double a,
                   double g, hipStream_t st) {
  if (stream_ok(A.n, sizeof(T))) {
    stream_smooth<T>(A, x, xprev, b, xout, a, g, st);
    return;
  }
  const Geo G = make_geo(A.n);
  if (A.op == 0)
    LAUNCH_B((k_smooth<0, T>), ew_blocks(G.npts), st, A, G, x, xprev, b, xout, a, g,
             batch_args());
  else if (A.op == 2)
    LAUNCH_B((k_smooth<2, T>), ew_blocks(G.npts), st, A, G, x, xprev, b, xout, a, g,
             batch_args());
  else
    LAUNCH_B((k_smooth<1, T>), ew_blocks(G.npts), st, A, G, x, xprev, b, xout, a, g,
             batch_args());
}
template void launch_smooth<double>(const OpDesc&, const double*, const double*, const double*,
                                    double*, double, double, hipStream_t);
template void launch_smooth<float>(const OpDesc&, const float*, const float*, const float*,
                                   float*, double, double, hipStream_t);

template <typename T>
void launch_smooth0(const OpDesc& A, const T* b, T* xout, double a, hipStream_t st) {
  const Geo G = make_geo(A.n);
  if (A.op == 0)
    LAUNCH_B((k_smooth0<0, T>), ew_blocks(G.npts), st, A, G, b, xout, a, batch_args());
  else if (A.op == 2)
    LAUNCH_B((k_smooth0<2, T>), ew_blocks(G.npts), st, A, G, b, xout, a, batch_args());
  else
    LAUNCH_B((k_smooth0<1, T>), ew_blocks(G.npts), st, A, G, b, xout, a, batch_args());
}
template void launch_smooth0<double>(const OpDesc&, const double*, double*, double, hipStream_t);
template void launch_smooth0<float>(const OpDesc&, const float*, float*, double, hipStream_t);

void launch_jacobi_pc(const OpDesc& A, const double* r, double* z, hipStream_t st) {
  const Geo G = make_geo(A.n);
  if (A.op == 0)
    LAUNCH(k_jacobi_pc<0>, ew_blocks(G.npts), st, A, G, r, z);
  else if (A.op == 2)
    LAUNCH(k_jacobi_pc<2>, ew_blocks(G.npts), st, A, G, r, z);
  else
    LAUNCH(k_jacobi_pc<1>, ew_blocks(G.npts), st, A, G, r, z);
}

template <typename T>
void launch_restrict(int nf, const T* fine, T* coarse, hipStream_t st) {
  // (a batch of instances fills the GPU with tiles already from nf = 256)
  if (transfer_stream_ok(nf) || (batch_count() > 1 && nf >= 256)) {
    stream_restrict<T>(nf, fine, coarse, st);
    return;
  }
  const Geo F = make_geo(nf), C = make_geo(nf / 2);
  LAUNCH_B((k_restrict<T>), ew_blocks(C.npts), st, F, C, fine, coarse, batch_args());
}
template void launch_restrict<double>(int, const double*, double*, hipStream_t);
template void launch_restrict<float>(int, const float*, float*, hipStream_t);

template <typename T>
void launch_prolong_add(int nf, const T* coarse, T* fine, hipStream_t st) {
  if (transfer_stream_ok(nf) || (batch_count() > 1 && nf >= 256)) {
    stream_prolong_add<T>(nf, coarse, fine, st);
    return;
  }
  const Geo F = make_geo(nf), C = make_geo(nf / 2);
  LAUNCH_B((k_prolong_add<T>), ew_blocks(F.npts), st, F, C, coarse, fine, batch_args());
}
template void launch_prolong_add<double>(int, const double*, double*, hipStream_t);
template void launch_prolong_add<float>(int, const float*, float*, hipStream_t);

template <typename T>
void launch_coarse_solve(int size, const double* G, const T* b, T* x, hipStream_t st) {
  hipLaunchKernelGGL((k_coarse_solve<T>), dim3(1), dim3(64), 0, st, size, G, b, x);
}
template void launch_coarse_solve<double>(int, const double*, const double*, double*, hipStream_t);
template void launch_coarse_solve<float>(int, const double*, const float*, float*, hipStream_t);

void launch_to_float(int64_t count, const double* x, float* y, hipStream_t st) {
  LAUNCH(k_to_float, ew_blocks(count), st, count, x, y);
}

void launch_to_double(int64_t count, const float* x, double* y, hipStream_t st) {
  LAUNCH(k_to_double, ew_blocks(count), st, count, x, y);
}

void launch_finalize_flex(const double* partials, int nparts, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_flex, dim3(1), dim3(kFinTPB), 0, st, partials, nparts, scal);
}

void launch_dot(int n, const double* x, const double* y, double* partials, int nparts,
                hipStream_t st) {
  LAUNCH(k_dot, nparts, st, make_geo(n), x, y, partials);
}

void launch_wsum_diff(int n, const double* x, const double* y, double* partials, int nparts,
                      hipStream_t st) {
  LAUNCH(k_wsum_diff, nparts, st, make_geo(n), x, y, partials);
}

void launch_residual_norms(const double* scal, double csq, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_residual_norms, dim3(1), dim3(64), 0, st, scal, csq, out);
}

void launch_finalize(const double* partials, int nparts, double* scal, int mode, int slot, int n,
                     hipStream_t st, double* host, double hseq) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinTPB), 0, st, partials, nparts, scal, mode, slot,
                     (double)n * (double)n, host, hseq);
}

int launch_cg_p(const OpDesc& A, const double* z, const double* p_old, double* p_new, double* q,
                double* x, const double* scal, bool first, double* partials, int nparts,
                hipStream_t st) {
  if (stream_ok(A.n)) return stream_cg_p(A, z, p_old, p_new, q, x, scal, first, partials, st);
  const Geo G = make_geo(A.n);
  if (A.op == 0)
    LAUNCH(k_cg_p<0>, nparts, st, A, G, z, p_old, p_new, q, x, scal, first ? 1 : 0, partials);
  else if (A.op == 2)
    LAUNCH(k_cg_p<2>, nparts, st, A, G, z, p_old, p_new, q, x, scal, first ? 1 : 0, partials);
  else
    LAUNCH(k_cg_p<1>, nparts, st, A, G, z, p_old, p_new, q, x, scal, first ? 1 : 0, partials);
  return nparts;
}

void launch_r_update(int n, double* r, const double* q, const double* scal, double* partials,
                     int nparts, hipStream_t st, float* r32) {
  LAUNCH(k_r_update, nparts, st, make_geo(n), r, q, scal, partials, r32);
}

void launch_x_update(int n, double* x, const double* p, const double* scal, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_x_update<double>, ew_blocks(G.npts), st, G, x, p, scal);
}
void launch_x_update(int n, double* x, const float* p, const double* scal, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_x_update<float>, ew_blocks(G.npts), st, G, x, p, scal);
}

void launch_sub_mean(int n, const double* x, double* y, const double* scal, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_sub_mean, ew_blocks(G.npts), st, G, x, y, scal, 1.0);
}

void launch_x_accum(int n, double* x, const float* const* p, int m, const double* alpha,
                    hipStream_t st) {
  const Geo G = make_geo(n);
  const int64_t nquad = G.npts / 4;
  RingPtrs R{};
  for (int i = 0; i < m; ++i) R.p[i] = p[i];
  const int blocks = ew_blocks(nquad);
  switch (m) {
#define BF_XACC(M_) \
  case M_:          \
    LAUNCH(k_x_accum<M_>, blocks, st, nquad, x, R, alpha); \
    break;
    BF_XACC(1) BF_XACC(2) BF_XACC(3) BF_XACC(4) BF_XACC(5) BF_XACC(6) BF_XACC(7) BF_XACC(8)
    BF_XACC(9) BF_XACC(10) BF_XACC(11) BF_XACC(12) BF_XACC(13) BF_XACC(14) BF_XACC(15)
    BF_XACC(16)
#undef BF_XACC
    default:
      break;
  }
}

void launch_project_start(int n, const double* x, double* b, double* r, float* r32,
                          const double* scal, double* partials, int nparts, hipStream_t st) {
  LAUNCH(k_project_start, nparts, st, make_geo(n), x, b, r, r32, scal, partials);
}

void launch_add_mean(int n, const double* x, double* y, const double* scal, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_sub_mean, ew_blocks(G.npts), st, G, x, y, scal, -1.0);
}

void launch_fill(int64_t count, double* x, double v, hipStream_t st) {
  LAUNCH(k_fill, ew_blocks(count), st, count, x, v);
}

void launch_copy(int64_t count, const double* x, double* y, hipStream_t st) {
  LAUNCH(k_copy, ew_blocks(count), st, count, x, y);
}

void launch_copy2(int64_t count, const double* x, double* y, hipStream_t st) {
  const int64_t pairs = count / 2;
  LAUNCH(k_copy2, ew_blocks(pairs), st, pairs, reinterpret_cast<const double2*>(x),
         reinterpret_cast<double2*>(y));
}

void launch_fill_i32(int count, int32_t* x, int32_t v, hipStream_t st) {
  LAUNCH(k_fill_i32, 1, st, count, x, v);
}

void launch_ch_rhs(int n, const double* phi, const double* prev, const double* base, double* b,
                   double* mu_ws, double dtM, double inv_npoly, double chi, double lo, double hi,
                   int32_t* clamp_count, hipStream_t st) {
  const Geo G = make_geo(n);
  if (n >= kRhsCols) {
    RhsCoef C{dtM * (double)n * (double)n, inv_npoly, chi, lo, hi};
    const int strips = n / kRhsCols;
    const int rgroups = (n + 1 + kRhsRows - 1) / kRhsRows;
    hipLaunchKernelGGL(k_ch_rhs_tile, dim3(strips * rgroups, 1), dim3(kBlock), 0, st, G,
                       (int64_t)0, strips, phi, prev, base, b, C, nullptr, 0, clamp_count);
    return;
  }
  LAUNCH(k_mu, ew_blocks(G.npts), st, G, phi, prev, mu_ws, inv_npoly, chi, lo, hi, clamp_count);
  LAUNCH(k_lap_axpy, ew_blocks(G.npts), st, G, mu_ws, base, b, dtM * (double)n * (double)n);
}

void launch_ch_rhs_batch(int n, int count, int64_t stride, const double* phi, double* b,
                         const double* icoef, int icoef_stride, int32_t* clamp_counts,
                         hipStream_t st) {
  const Geo G = make_geo(n);
  const int strips = n / kRhsCols;
  const int rgroups = (n + 1 + kRhsRows - 1) / kRhsRows;
  hipLaunchKernelGGL(k_ch_rhs_tile, dim3(strips * rgroups, count), dim3(kBlock), 0, st, G, stride,
                     strips, phi, nullptr, phi, b, RhsCoef{}, icoef, icoef_stride, clamp_counts);
}

int launch_mob(int n, double c, const double* m, const double* x, const double* b, double* y,
               double* partials, int nparts, hipStream_t st) {
  const Geo G = make_geo(n);
  if (!b) {
    LAUNCH(k_mob<0>, ew_blocks(G.npts), st, G, c, m, x, nullptr, y, nullptr);
    return 0;
  }
  LAUNCH(k_mob<1>, nparts, st, G, c, m, x, b, y, partials);
  return nparts;
}

template <typename T>
void launch_mob_smooth(int n, double cs, const T* m, const T* x, const T* xprev, const T* b,
                       T* xout, double a, double g, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_mob_smooth<T>, ew_blocks(G.npts), st, G, T(cs), m, x, xprev, b, xout, T(a), T(g));
}
template <typename T>
void launch_mob_smooth0(int n, double cs, const T* m, const T* b, T* xout, double a0,
                        hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_mob_smooth0<T>, ew_blocks(G.npts), st, G, T(cs), m, b, xout, T(a0));
}
template <typename T>
void launch_mob_residual(int n, double cs, const T* m, const T* x, const T* b, T* r,
                         hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_mob_residual<T>, ew_blocks(G.npts), st, G, T(cs), m, x, b, r);
}
template <typename T>
void launch_inject(int nf, const T* fine, T* coarse, hipStream_t st) {
  const Geo F = make_geo(nf), C = make_geo(nf / 2);
  LAUNCH(k_inject<T>, ew_blocks(C.npts), st, F, C, fine, coarse);
}
#define BF_MOB_INST(T)                                                                         \
  template void launch_mob_smooth<T>(int, double, const T*, const T*, const T*, const T*, T*,   \
                                     double, double, hipStream_t);                             \
  template void launch_mob_smooth0<T>(int, double, const T*, const T*, T*, double, hipStream_t); \
  template void launch_mob_residual<T>(int, double, const T*, const T*, const T*, T*,          \
                                       hipStream_t);                                           \
  template void launch_inject<T>(int, const T*, T*, hipStream_t);
BF_MOB_INST(double)
BF_MOB_INST(float)
#undef BF_MOB_INST

void launch_mob_rhs(int n, const double* phi, double* m, double* mu_ws, double* b, double M,
                    double dt, double inv_npoly, double chi, double lo, double hi,
                    int32_t* clamp_count, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_mu, ew_blocks(G.npts), st, G, phi, nullptr, mu_ws, inv_npoly, chi, lo, hi, clamp_count);
  LAUNCH(k_mob_field, ew_blocks(G.npts), st, G, phi, m, M, lo, hi);
  LAUNCH(k_mob_rhs, ew_blocks(G.npts), st, G, phi, mu_ws, m, b, dt * (double)n * (double)n);
}

void launch_divergence(int n, const double* u, const double* v, double* rhs, double scale,
                       hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_divergence, ew_blocks(G.npts), st, G, u, v, rhs, scale);
}

void launch_velocity(int n, const double* p, const double* us, const double* vs, double* u,
                     double* v, double scale, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_velocity, ew_blocks(G.npts), st, G, p, us, vs, u, v, scale);
}

void launch_momentum_rhs(int n, const double* u, const double* v, double dt, double e, double U,
                         double* bu, double* bv, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_momentum_rhs, ew_blocks(G.npts), st, G, u, v, dt, e, U, bu, bv);
}

void launch_advect_sub(int n, const double* phi, const double* u, const double* v, double* b,
                       double dt, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_advect_sub, ew_blocks(G.npts), st, G, phi, u, v, b, dt * 0.5 * (double)n);
}

void launch_wscale(int n, const double* x, double* y, bool inverse, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_wscale, ew_blocks(G.npts), st, G, x, y, inverse ? 1 : 0);
}

void launch_adjoint_rhs(int n, const double* e, const double* phi, const double* u,
                        const double* v, const double* du, const double* dv, double* lam,
                        const AdjCoef& C, double* partials, int nparts, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_adjoint_rhs, nparts, st, G, e, phi, u, v, du, dv, lam, C, partials);
}

void launch_mdot(int n, const double* V, int m, const double* w, double* partials, int nparts,
                 hipStream_t st) {
  const Geo G = make_geo(n);
  for (int k0 = 0; k0 < m; k0 += kMdotGroup) LAUNCH(k_mdot, nparts, st, G, V, m, k0, w, partials);
}

void launch_finalize_multi(const double* partials, int nparts, int m, double* scal, int slot,
                           hipStream_t st) {
  LAUNCH(k_finalize_multi, m, st, partials, nparts, scal, slot);
}

void launch_maxpy(int n, const double* V, int m, const double* h, double* w, double* partials,
                  int nparts, hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_maxpy, partials ? nparts : ew_blocks(G.npts), st, G, V, m, h, w, partials);
}

void launch_axpy_multi(int n, const double* Z, int m, const double* y, double* x,
                       hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_axpy_multi, ew_blocks(G.npts), st, G, Z, m, y, x);
}

void launch_scale(int n, const double* x, double* y, const double* scal, int slot, int invert_sqrt,
                  hipStream_t st) {
  const Geo G = make_geo(n);
  LAUNCH(k_scale, ew_blocks(G.npts), st, G, x, y, scal, slot, invert_sqrt);
}

}  // namespace bf
