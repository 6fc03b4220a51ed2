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

// Fields are addressed by their offset into the LDS array, never through
// pointers kept in arrays indexed at run time: the compiler could not tell
// that such a pointer is an LDS address and would access it with generic
// (flat) loads and stores, which take the slower path of global memory
// instructions (measured with a 64 x 64 top level: float64 tail 88 us that
// way against 43 us with LDS instructions, float32 49 against 40).
__device__ __forceinline__ int log2_of(int n) {
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  return lg;
}

// Calls f(j, i) for every node of an (n+1) x n level (n <= 64, a power of
// two): thread t takes column i = t mod n of rows t / n, t / n + 1024 / n, ...
// The column arithmetic is then loop-invariant, and with n = 64 every
// wavefront covers exactly one row, so the row index and everything derived
// from it (reflection, row offsets, row coefficients) stays in scalar
// registers.  The tail runs on one CU and is bound by vector instructions.
template <typename F>
__device__ __forceinline__ void for_nodes(int n, int lg, F f) {
  const int i = threadIdx.x & (n - 1);
  const int jstep = kTailThreads >> lg;
  if (n >= 64) {
    for (int j = __builtin_amdgcn_readfirstlane(threadIdx.x >> lg); j <= n; j += jstep) f(j, i);
  } else {
    for (int j = threadIdx.x >> lg; j <= n; j += jstep) f(j, i);
  }
}

// Stencil values around (i, j) of an LDS field (rows reflected, columns
// wrapped), with row offsets by shifts (n = 2^lg).
template <int OP, typename T>
__device__ __forceinline__ Nb13T<T> tail_gather(const T* x, int i, int j, int n, int lg) {
  const int mask = n - 1;
  const T* r0 = x + (j << lg);
  const T* rm1 = x + (refl(j - 1, n) << lg);
  const T* rp1 = x + (refl(j + 1, n) << lg);
  const int im1 = (i - 1) & mask, ip1 = (i + 1) & mask;
  Nb13T<T> v;
  v.c = r0[i];
  v.xm1 = r0[im1];
  v.xp1 = r0[ip1];
  v.ym1 = rm1[i];
  v.yp1 = rp1[i];
  if (OP == 1) {
    const T* rm2 = x + (refl(j - 2, n) << lg);
    const T* rp2 = x + (refl(j + 2, n) << lg);
    v.dmm = rm1[im1];
    v.dmp = rm1[ip1];
    v.dpm = rp1[im1];
    v.dpp = rp1[ip1];
    v.xm2 = r0[(i - 2) & mask];
    v.xp2 = r0[(i + 2) & mask];
    v.ym2 = rm2[i];
    v.yp2 = rp2[i];
  }
  return v;
}

// The 64 x 64 level (65 rows) with each thread on four consecutive rows of
// one column (rows 4 w .. 4 w + 3 for wavefront w; the last wavefront also
// takes row 64): the column's values of the rows in reach are read from LDS
// once into registers and shared by the thread's nodes, 7 reads per node
// instead of 13 for the 13-point stencil.  scale(jr) multiplies every value
// read from row jr (the first iterate formed from b); f(j, idx, v) receives
// each node's stencil values.
template <int OP, typename T, typename S, typename F>
__device__ __forceinline__ void for_nodes64(const T* X, S scale, F f) {
  constexpr int n = 64, lg = 6;
  const int i = threadIdx.x & (n - 1);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> lg));
  const int j0 = 4 * w;
  const int nr = w == (kTailThreads >> lg) - 1 ? 5 : 4;
  const int im1 = (i - 1) & (n - 1), ip1 = (i + 1) & (n - 1);
  const int im2 = (i - 2) & (n - 1), ip2 = (i + 2) & (n - 1);
  constexpr int R = OP == 1 ? 2 : 1;
  // column i: rows j0-R .. j0+nr-1+R; columns i-1, i+1: rows j0-1 .. j0+nr (OP 1)
  // or j0 .. j0+nr-1; columns i-2, i+2: rows j0 .. j0+nr-1 (OP 1)
  T cc[5 + 2 * R], cm1[7], cp1[7], cm2[5], cp2[5];
#pragma unroll
  for (int r = 0; r < 5 + 2 * R; ++r) {
    if (r < nr + 2 * R) {
      const int jr = refl(j0 - R + r, n);
      cc[r] = X[(jr << lg) + i] * scale(jr);
    }
  }
  constexpr int R1 = OP == 1 ? 1 : 0;
#pragma unroll
  for (int r = 0; r < 5 + 2 * R1; ++r) {
    if (r < nr + 2 * R1) {
      const int jr = refl(j0 - R1 + r, n);
      const T sc = scale(jr);
      cm1[r] = X[(jr << lg) + im1] * sc;
      cp1[r] = X[(jr << lg) + ip1] * sc;
    }
  }
  if constexpr (OP == 1) {
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      if (r < nr) {
        const int jr = j0 + r;
        const T sc = scale(jr);
        cm2[r] = X[(jr << lg) + im2] * sc;
        cp2[r] = X[(jr << lg) + ip2] * sc;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    if (s < nr) {
      Nb13T<T> v;
      v.c = cc[s + R];
      v.ym1 = cc[s + R - 1];
      v.yp1 = cc[s + R + 1];
      v.xm1 = cm1[s + R1];
      v.xp1 = cp1[s + R1];
      if constexpr (OP == 1) {
        v.ym2 = cc[s];
        v.yp2 = cc[s + 4];
        v.dmm = cm1[s];
        v.dmp = cp1[s];
        v.dpm = cm1[s + 2];
        v.dpp = cp1[s + 2];
        v.xm2 = cm2[s];
        v.xp2 = cp2[s];
      }
      const int j = j0 + s;
      f(j, (j << lg) + i, v);
    }
  }
}

// xout = x + a D^{-1} (b - A x) + g (x - xprev)  (xprev = -1: no xprev term;
// xprev = kPrevFromB: xprev is the first iterate a0 D^{-1} b, formed from b)
constexpr int kPrevFromB = -2;
template <int OP, typename T>
__device__ void tail_sweep(T* lds, const TailLevel& L, int x, int xprev, int b, int xout,
                           double a, double g) {
  const int n = L.n, lg = log2_of(n);
  const T ta = T(a), tg = T(g);
  const bool hp = xprev >= 0, pb = xprev == kPrevFromB;
  const T* X = lds + x;
  const T* XP = lds + (hp ? xprev : x);
  const T* B = lds + b;
  T* O = lds + xout;
  auto node = [&](int j, int idx, const Nb13T<T>& v) {
    const T ax = apply_vals<OP>(v, T(row_coef<OP>(L.coef, j, n)));
    const T ad = ta * T(row_dinv<OP>(L.dinv_int, L.dinv_edge, j, n));
    const T prev = hp ? XP[idx]
                      : pb ? T(L.a[0] * row_dinv<OP>(L.dinv_int, L.dinv_edge, j, n)) * B[idx]
                           : T(0);
    O[idx] = v.c + ad * (B[idx] - ax) + tg * (v.c - prev);
  };
  if (n == 64) {
    for_nodes64<OP, T>(X, [](int) { return T(1); }, node);
  } else {
    for_nodes(n, lg, [&](int j, int i) {
      const int idx = (j << lg) + i;
      node(j, idx, tail_gather<OP>(X, i, j, n, lg));
    });
  }
  __syncthreads();
}

// The first sweep from a zero iterate, x2 = x1 + a1 D^{-1} (b - A x1) + g1 x1,
// with x1 = a0 D^{-1} b formed where it is read, which saves the phase that
// would store x1 (the products may be contracted into the stencil's sums, so
// the result can differ from the stored-x1 form by rounding).
template <int OP, typename T>
__device__ void tail_sweep_from_b(T* lds, const TailLevel& L, int b, int xout) {
  const int n = L.n, lg = log2_of(n);
  const T a1 = T(L.a[1]), g1 = T(L.g[1]);
  const T* B = lds + b;
  T* O = lds + xout;
  auto x1 = [&](int jr) -> T { return T(L.a[0] * row_dinv<OP>(L.dinv_int, L.dinv_edge, jr, n)); };
  auto node = [&](int j, int idx, const Nb13T<T>& v) {
    const T ax = apply_vals<OP>(v, T(row_coef<OP>(L.coef, j, n)));
    const T ad = a1 * T(row_dinv<OP>(L.dinv_int, L.dinv_edge, j, n));
    O[idx] = v.c + ad * (B[idx] - ax) + g1 * v.c;
  };
  if (n == 64) {
    for_nodes64<OP, T>(B, x1, node);
    __syncthreads();
    return;
  }
  for_nodes(n, lg, [&](int j, int i) {
    const int idx = (j << lg) + i;
    Nb13T<T> v = tail_gather<OP>(B, i, j, n, lg);
    const T s0 = x1(j), sm1 = x1(refl(j - 1, n)), sp1 = x1(refl(j + 1, n));
    v.c *= s0;
    v.xm1 *= s0;
    v.xp1 *= s0;
    v.ym1 *= sm1;
    v.yp1 *= sp1;
    if (OP == 1) {
      const T sm2 = x1(refl(j - 2, n)), sp2 = x1(refl(j + 2, n));
      v.xm2 *= s0;
      v.xp2 *= s0;
      v.dmm *= sm1;
      v.dmp *= sm1;
      v.dpm *= sp1;
      v.dpp *= sp1;
      v.ym2 *= sm2;
      v.yp2 *= sp2;
    }
    node(j, idx, v);
  });
  __syncthreads();
}

template <int OP, typename T>
__device__ void tail_body(const TailArgs& P, const T* b_in, T* x_out) {
  __shared__ T lds[kTailMaxDoubles];
  const int tid = threadIdx.x;
  // LDS offsets of each level's fields
  int xa[kTailMaxLevels], xb[kTailMaxLevels], bb[kTailMaxLevels];
  int off = 0;
  for (int l = 0; l < P.nlev; ++l) {
    const int npts = (P.lev[l].n + 1) * P.lev[l].n;
    xa[l] = off;
    xb[l] = off + npts;
    bb[l] = off + 2 * npts;
    off += 3 * npts;
  }
  const int xc = off;       // coarsest x (20)
  const int bc = off + 20;  // coarsest b (20)

  // right-hand side of the top tail level: every thread's loads issued
  // together (clamped to the field), then stored to LDS
  {
    const int npts = (P.lev[0].n + 1) * P.lev[0].n;
    T* B = lds + bb[0];
    constexpr int kPer = (65 * 64 + kTailThreads - 1) / kTailThreads;
    T v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) v[r] = b_in[min(tid + r * kTailThreads, npts - 1)];
#pragma unroll
    for (int r = 0; r < kPer; ++r)
      if (tid + r * kTailThreads < npts) B[tid + r * kTailThreads] = v[r];
  }
  __syncthreads();

  int res[kTailMaxLevels];  // field holding each level's iterate
  int oth[kTailMaxLevels];
  // downward leg
  for (int l = 0; l < P.nlev; ++l) {
    const TailLevel& L = P.lev[l];
    const int n = L.n, lg = log2_of(n);
    int cur = xa[l];
    int o = xb[l];
    if (L.degree >= 2) {
      // x1 = a0 D^{-1} b is never stored: the first sweep and (as x_prev) the
      // second form it from b (64 x 64 tail level with CH, float32: 43 -> 37 us)
      tail_sweep_from_b<OP, T>(lds, L, bb[l], o);
      cur = xb[l];
      o = xa[l];
      for (int k = 2; k < L.degree; ++k) {
        const int prev = L.g[k] == 0.0 ? -1 : (k == 2 ? kPrevFromB : o);
        tail_sweep<OP, T>(lds, L, cur, prev, bb[l], o, L.a[k], L.g[k]);
        const int t = cur;
        cur = o;
        o = t;
      }
    } else {
      T* C = lds + cur;
      const T* B = lds + bb[l];
      for_nodes(n, lg, [&](int j, int i) {
        const int idx = (j << lg) + i;
        C[idx] = T(L.a[0] * row_dinv<OP>(L.dinv_int, L.dinv_edge, j, n)) * B[idx];
      });
      __syncthreads();
    }
    // residual, into the iterate buffer the sweeps are done with
    {
      const T* C = lds + cur;
      const T* B = lds + bb[l];
      T* R = lds + o;
      auto node = [&](int j, int idx, const Nb13T<T>& v) {
        R[idx] = B[idx] - apply_vals<OP>(v, T(row_coef<OP>(L.coef, j, n)));
      };
      if (n == 64) {
        for_nodes64<OP, T>(C, [](int) { return T(1); }, node);
      } else {
        for_nodes(n, lg, [&](int j, int i) {
          const int idx = (j << lg) + i;
          node(j, idx, tail_gather<OP>(C, i, j, n, lg));
        });
      }
    }
    __syncthreads();
    // restriction to the next level (or to the coarsest grid)
    {
      const int nc = n / 2, cpts = (nc + 1) * nc, lgc = lg - 1;
      const T* R = lds + o;
      T* BN = lds + ((l + 1 < P.nlev) ? bb[l + 1] : bc);
      for (int idx = tid; idx < cpts; idx += kTailThreads) {
        const int I = idx & (nc - 1), J = idx >> lgc;
        BN[idx] = restrict_at(R, n, n - 1, I, J);
      }
    }
    __syncthreads();
    res[l] = cur;
    oth[l] = o;
  }
  // coarsest grid: x = G b
  if (tid < 20) {
    double acc = 0.0;
    for (int k = 0; k < 20; ++k) acc += P.G[tid * 20 + k] * double(lds[bc + k]);
    lds[xc + tid] = T(acc);
  }
  __syncthreads();
  // upward leg
  for (int l = P.nlev - 1; l >= 0; --l) {
    const TailLevel& L = P.lev[l];
    const int n = L.n, npts = (n + 1) * n, nc = n / 2, lg = log2_of(n);
    int cur = res[l];
    int o = oth[l];
    {
      const T* E = lds + ((l + 1 < P.nlev) ? res[l + 1] : xc);
      T* C = lds + cur;
      for (int idx = tid; idx < npts; idx += kTailThreads) {
        const int i = idx & (n - 1), j = idx >> lg;
        C[idx] += prolong_at(E, nc, nc - 1, i, j);
      }
    }
    __syncthreads();
    for (int k = 0; k < L.degree; ++k) {
      tail_sweep<OP, T>(lds, L, cur, L.g[k] != 0.0 ? o : -1, bb[l], o, L.a[k], L.g[k]);
      const int t = cur;
      cur = o;
      o = t;
    }
    res[l] = cur;
  }
  {
    const int npts = (P.lev[0].n + 1) * P.lev[0].n;
    const T* C = lds + res[0];
    for (int idx = tid; idx < npts; idx += kTailThreads) x_out[idx] = C[idx];
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
