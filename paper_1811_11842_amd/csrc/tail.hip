// Coarse tail of the V-cycle: every level with n <= 64 (down to the exact
// solve on the 5 x 4 grid) runs inside one workgroup of 1024 threads, with all
// fields of those levels resident in LDS (134 KB in float64, of the 160 KB of
// a CU).  On these levels a separate launch per sweep would cost far more
// than the arithmetic (each grid is at most 65 x 64 nodes), so the whole lower
// part of the cycle is a single launch whose phases are separated by
// workgroup barriers.
//
// The operations are those of the global-memory kernels (same device
// helpers): the polynomial smoother, the residual, R and P, and x = G b on the
// coarsest grid.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"
#include "stencil_ops.hpp"

namespace bf {

constexpr int kTailThreads = 1024;

// LDS layout: for each smoothing level (n = top, top/2, ..., 8) three arrays
// xa, xb, b of (n+1) n elements, then the coarsest x and b (20 each).  The
// residual of the downward leg goes into whichever of xa, xb the
// pre-smoothing no longer needs (the first post-smoothing sweep, with
// Chebyshev coefficient g = 0, does not read it).
__host__ __device__ inline int tail_lds_doubles(int top) {
  int total = 0;
  for (int n = top; n > 4; n /= 2) total += 3 * (n + 1) * n;
  return total + 2 * 20;
}
static_assert(kTailMaxDoubles >= 3 * (65 * 64 + 33 * 32 + 17 * 16 + 9 * 8) + 40,
              "tail LDS too small for its top level");

template <int OP, typename T>
__device__ void tail_sweep(const TailLevel& L, const T* x, const T* xprev, const T* b, T* xout,
                           double a, double g) {
  const int n = L.n, mask = n - 1, npts = (n + 1) * n;
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  const T ta = T(a), tg = T(g);
  for (int idx = threadIdx.x; idx < npts; idx += kTailThreads) {
    const int i = idx & mask, j = idx >> lg;
    const Nb13T<T> v = gather<OP>(x, i, j, n, mask);
    const T ax = apply_vals<OP>(v, T(row_coef<OP>(L.coef, j, n)));
    const T dinv = T(row_dinv<OP>(L.dinv_int, L.dinv_edge, j, n));
    const T prev = xprev ? xprev[idx] : T(0);
    xout[idx] = v.c + ta * dinv * (b[idx] - ax) + tg * (v.c - prev);
  }
  __syncthreads();
}

template <int OP, typename T>
__device__ void tail_body(const TailArgs& P, const T* b_in, T* x_out) {
  __shared__ T lds[kTailMaxDoubles];
  const int tid = threadIdx.x;
  // carve LDS
  T* xa[kTailMaxLevels];
  T* xb[kTailMaxLevels];
  T* bb[kTailMaxLevels];
  int off = 0;
  for (int l = 0; l < P.nlev; ++l) {
    const int npts = (P.lev[l].n + 1) * P.lev[l].n;
    xa[l] = lds + off;
    xb[l] = xa[l] + npts;
    bb[l] = xb[l] + npts;
    off += 3 * npts;
  }
  T* xc = lds + off;  // coarsest x (20)
  T* bc = xc + 20;    // coarsest b (20)

  // right-hand side of the top tail level
  {
    const int npts = (P.lev[0].n + 1) * P.lev[0].n;
    for (int idx = tid; idx < npts; idx += kTailThreads) bb[0][idx] = b_in[idx];
  }
  __syncthreads();

  T* res[kTailMaxLevels];  // buffer holding each level's iterate
  T* oth[kTailMaxLevels];
  // downward leg
  for (int l = 0; l < P.nlev; ++l) {
    const TailLevel& L = P.lev[l];
    const int n = L.n, npts = (n + 1) * n;
    T* cur = xa[l];
    T* o = xb[l];
    for (int idx = tid; idx < npts; idx += kTailThreads) {
      const int j = idx / n;
      const double dinv = row_dinv<OP>(L.dinv_int, L.dinv_edge, j, n);
      cur[idx] = T(L.a[0] * dinv) * bb[l][idx];
    }
    __syncthreads();
    for (int k = 1; k < L.degree; ++k) {
      tail_sweep<OP, T>(L, cur, (k == 1 || L.g[k] == 0.0) ? nullptr : o, bb[l], o, L.a[k],
                        L.g[k]);
      T* t = cur;
      cur = o;
      o = t;
    }
    // residual, into the iterate buffer the sweeps are done with
    T* rl = o;
    for (int idx = tid; idx < npts; idx += kTailThreads) {
      const int i = idx & (n - 1), j = idx / n;
      const Nb13T<T> v = gather<OP>(cur, i, j, n, n - 1);
      rl[idx] = bb[l][idx] - apply_vals<OP>(v, T(row_coef<OP>(L.coef, j, n)));
    }
    __syncthreads();
    // restriction to the next level (or to the coarsest grid)
    const int nc = n / 2, cpts = (nc + 1) * nc;
    T* bnext = (l + 1 < P.nlev) ? bb[l + 1] : bc;
    for (int idx = tid; idx < cpts; idx += kTailThreads) {
      const int I = idx & (nc - 1), J = idx / nc;
      bnext[idx] = restrict_at(rl, n, n - 1, I, J);
    }
    __syncthreads();
    res[l] = cur;
    oth[l] = o;
  }
  // coarsest grid: x = G b
  if (tid < 20) {
    double acc = 0.0;
    for (int k = 0; k < 20; ++k) acc += P.G[tid * 20 + k] * double(bc[k]);
    xc[tid] = T(acc);
  }
  __syncthreads();
  // upward leg
  for (int l = P.nlev - 1; l >= 0; --l) {
    const TailLevel& L = P.lev[l];
    const int n = L.n, npts = (n + 1) * n, nc = n / 2;
    const T* e = (l + 1 < P.nlev) ? res[l + 1] : xc;
    T* cur = res[l];
    T* o = oth[l];
    for (int idx = tid; idx < npts; idx += kTailThreads) {
      const int i = idx & (n - 1), j = idx / n;
      cur[idx] += prolong_at(e, nc, nc - 1, i, j);
    }
    __syncthreads();
    for (int k = 0; k < L.degree; ++k) {
      tail_sweep<OP, T>(L, cur, L.g[k] != 0.0 ? o : nullptr, bb[l], o, L.a[k], L.g[k]);
      T* t = cur;
      cur = o;
      o = t;
    }
    res[l] = cur;
  }
  {
    const int npts = (P.lev[0].n + 1) * P.lev[0].n;
    for (int idx = tid; idx < npts; idx += kTailThreads) x_out[idx] = res[0][idx];
  }
}

template <int OP, typename T>
__global__ void __launch_bounds__(kTailThreads) k_tail(TailArgs P, const T* b_in, T* x_out) {
  tail_body<OP, T>(P, b_in, x_out);
}

// One workgroup per instance of a batch; args[i] holds instance i's levels.
template <int OP, typename T>
__global__ void __launch_bounds__(kTailThreads) k_tail_batch(const TailArgs* args, const T* b_in,
                                                             T* x_out, int64_t sin,
                                                             int64_t sout) {
  const int i = blockIdx.x;
  tail_body<OP, T>(args[i], b_in + (int64_t)i * sin, x_out + (int64_t)i * sout);
}

template <typename T>
void launch_tail_batch(int op, const TailArgs* args, int count, const T* b_in, T* x_out,
                       int64_t sin, int64_t sout, hipStream_t st) {
  if (op == 0)
    hipLaunchKernelGGL((k_tail_batch<0, T>), dim3(count), dim3(kTailThreads), 0, st, args, b_in,
                       x_out, sin, sout);
  else if (op == 2)
    hipLaunchKernelGGL((k_tail_batch<2, T>), dim3(count), dim3(kTailThreads), 0, st, args, b_in,
                       x_out, sin, sout);
  else
    hipLaunchKernelGGL((k_tail_batch<1, T>), dim3(count), dim3(kTailThreads), 0, st, args, b_in,
                       x_out, sin, sout);
}
template void launch_tail_batch<double>(int, const TailArgs*, int, const double*, double*,
                                        int64_t, int64_t, hipStream_t);

template <typename T>
void launch_tail(int op, const TailArgs& P, const T* b_in, T* x_out, hipStream_t st) {
  if (op == 0)
    hipLaunchKernelGGL((k_tail<0, T>), dim3(1), dim3(kTailThreads), 0, st, P, b_in, x_out);
  else if (op == 2)
    hipLaunchKernelGGL((k_tail<2, T>), dim3(1), dim3(kTailThreads), 0, st, P, b_in, x_out);
  else
    hipLaunchKernelGGL((k_tail<1, T>), dim3(1), dim3(kTailThreads), 0, st, P, b_in, x_out);
}
template void launch_tail<double>(int, const TailArgs&, const double*, double*, hipStream_t);
template void launch_tail<float>(int, const TailArgs&, const float*, float*, hipStream_t);

}  // namespace bf
