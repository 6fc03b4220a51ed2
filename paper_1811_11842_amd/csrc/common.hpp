// Shared device helpers: grid indexing with periodic x and reflected y,
// trapezoid weights, deterministic block reductions.
//
// Grid convention (Sec. 4 of the paper): n intervals per side, nodes
// (i*h, j*h); x periodic (columns 0..n-1), y rows 0..n with two ghost layers
// given by even reflection (eq. discreteBC): row -k is row k, row n+k is row
// n-k.  Fields are row-major (n+1) x n float64, x fastest.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bf {

constexpr int kBlock = 256;          // threads per block (4 wave64)
constexpr int kMaxRedBlocks = 1024;  // partial sums per reduction

// Scalar slots of the per-grid device scalar array.
enum Slot {
  S_BN2 = 0,   // ||b||_W^2
  S_RZ = 1,    // <r, z>_W of the current iteration
  S_RZOLD = 2, // previous <r, z>_W
  S_PQ = 3,    // <p, A p>_W
  S_ALPHA = 4, // rz / pq
  S_BETA = 5,  // rz / rzold
  S_RR = 6,    // ||r||_W^2 (recursive residual)
  S_MEAN = 7,  // weighted mean of the last reduced field
  S_RTRUE = 8, // ||b - A x||_W^2
  S_TMP = 9,
  S_ULP2 = 10, // sum_W ulp(x)^2 (representation floor estimate)
  S_GB = 11,   // initial guess: <b, A x0>_W
  S_GG = 12,   // initial guess: <A x0, A x0>_W
  S_GAMMA = 13,  // initial guess: its scale factor
  S_GM = 16,   // GMRES scalars start here (up to 64+ slots)
  S_AHIST = 224,  // CG: alpha of the steps whose iterate update is pending (kRing slots)
  S_HSEQ = 250,   // pinned host scalars only: sequence number of the last value mirrored there
  kNumSlots = 256
};
// Search directions of CG kept for one batched iterate update (float32 CG).
constexpr int kRing = 16;

enum FinalizeMode {
  F_STORE = 0,   // scal[slot] = sum
  F_ALPHA = 1,   // scal[S_PQ] = sum; scal[S_ALPHA] = scal[S_RZ] / sum (also into scal[slot] if slot > 0)
  F_BETA = 2,    // scal[S_RZOLD] = scal[S_RZ]; scal[S_RZ] = sum; beta = sum / rzold
  F_MEAN = 3     // scal[S_MEAN] = sum / (n*n)
};

struct Geo {
  int n;       // intervals (columns)
  int log2n;
  int mask;    // n - 1
  int64_t npts;  // (n+1) * n
};

__host__ __device__ inline Geo make_geo(int n) {
  Geo g;
  g.n = n;
  int l = 0;
  while ((1 << l) < n) ++l;
  g.log2n = l;
  g.mask = n - 1;
  g.npts = (int64_t)(n + 1) * n;
  return g;
}

// Even reflection of a row index into 0..n (valid for -n <= j <= 2n).
__device__ __forceinline__ int refl(int j, int n) {
  j = j < 0 ? -j : j;
  return j > n ? 2 * n - j : j;
}

__device__ __forceinline__ double row_weight(int j, int n) {
  return (j == 0 || j == n) ? 0.5 : 1.0;
}

// Sum over a 256-thread block; result valid in thread 0.  Fixed order, so
// the value is reproducible bit for bit.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += part[w];
  }
  __syncthreads();
  return t;
}

// Sum over a block of NT threads (NT a multiple of 64); result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v) {
  __shared__ double part[NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += part[w];
  }
  __syncthreads();
  return t;
}

inline int red_blocks(int64_t npts) {
  int64_t b = (npts + kBlock - 1) / kBlock;
  return (int)(b < kMaxRedBlocks ? b : kMaxRedBlocks);
}

inline int ew_blocks(int64_t npts) {
  int64_t b = (npts + kBlock - 1) / kBlock;
  const int64_t cap = 65536;
  return (int)(b < cap ? b : cap);
}

}  // namespace bf
