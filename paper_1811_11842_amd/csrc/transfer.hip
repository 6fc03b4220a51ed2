// Grid-transfer kernels for the large levels (fine grid n_f >= 256).
//
// Cubic interpolation P and its weighted adjoint R = 1/4 W_c^-1 P^T W_f
// (tensor products of the 1-D weights (-1, 9, 16, 9, -1)/16 and
// {0: 1/2, +-1: 9/32, +-3: -1/32}), periodic in x, even reflection in y.
//
// Same tiling as the stencil kernels: every wavefront owns a tile of CR
// coarse rows by 128 coarse columns (256 fine columns), each lane two coarse
// columns I0 = c/2, I0 + 1 and the four fine columns c .. c+3 between them.
// All rows of the tile are loaded at once; the neighbouring columns come from
// the adjacent lanes by DPP wave shifts, lanes 0 and 63 load the columns
// beyond the wavefront's edge (periodic wrap).  Tiles are numbered
// row-group-major, so the resident wavefronts cover one compact band of rows.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace bf {

namespace {

constexpr int kTPB = 256;
constexpr int kCR = 4;              // coarse rows per tile
constexpr int kMaxBlocks = 16384;   // beyond this, wavefronts loop over tiles

template <typename T, int N>
struct alignas(sizeof(T) * N) Vec {
  T v[N];
};

__device__ __forceinline__ float shl_in(float v) {  // lane i <- lane i-1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float shr_in(float v) {  // lane i <- lane i+1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double shl_in(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double shr_in(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

struct TArgs {
  int nf, nc;
  int wstrips, tiles;
  int bpi;              // workgroups per instance (batches)
  int64_t sf, sc;       // fine / coarse stride between instances
};

// coarse = R fine.  Per fine row f the lane forms the x-restricted values
// rs(f, I) = 1/2 r(f,2I) + 9/32 (r(f,2I-1) + r(f,2I+1)) - 1/32 (r(f,2I-3) + r(f,2I+3))
// for I = I0, I0+1; coarse(J, I) combines rs over fine rows 2J-3 .. 2J+3
// (reflected) with the same weights.
template <typename T>
__global__ void __launch_bounds__(kTPB) k_restrict_tile(TArgs A, const T* __restrict__ fine,
                                                        T* __restrict__ coarse) {
  constexpr int NF = 2 * kCR + 5;
  const int nf = A.nf, nc = A.nc, fmask = nf - 1;
  const int lane = threadIdx.x & 63;
  const bool hl = lane == 0, hr = lane == 63;
  const T h = T(0.5), w1 = T(9.0 / 32), w3 = T(-1.0 / 32);
  const int inst = blockIdx.x / A.bpi;
  fine += (int64_t)inst * A.sf;
  coarse += (int64_t)inst * A.sc;
  for (int t = (blockIdx.x - inst * A.bpi) * (kTPB / 64) + (threadIdx.x >> 6); t < A.tiles;
       t += A.bpi * (kTPB / 64)) {
    const int rg = t / A.wstrips;
    const int strip = t - rg * A.wstrips;
    const int J0 = rg * kCR;
    const int Jl = min(J0 + kCR, nc + 1) - 1;
    const int c = strip * 256 + 4 * lane;  // fine columns c .. c+3
    const int hcol = hl ? ((c - 4) & fmask) : ((c + 4) & fmask);
    // every load of the tile first (their latencies overlap): the fine rows
    // 2 J0 - 3 .. 2 Jl + 3 (reflected; rows a short last tile does not reach
    // repeat row 2 Jl + 3 and are unused), then the halo columns of lanes 0
    // and 63 (lane 0: columns c-3, c-1; lane 63: column c+5)
    Vec<T, 4> fo[NF];
    T e0[NF], e1[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const T* row = fine + (int64_t)refl(min(2 * J0 - 3 + k, 2 * Jl + 3), nf) * nf;
      fo[k] = *reinterpret_cast<const Vec<T, 4>*>(row + c);
      e0[k] = e1[k] = T(0);
    }
    if (hl || hr) {
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        const T* row = fine + (int64_t)refl(min(2 * J0 - 3 + k, 2 * Jl + 3), nf) * nf;
        const Vec<T, 4> hv = *reinterpret_cast<const Vec<T, 4>*>(row + hcol);
        e0[k] = hv.v[1];
        e1[k] = hv.v[3];
      }
    }
    T rs0[NF], rs1[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const Vec<T, 4>& o = fo[k];
      T l1 = shl_in(o.v[3]), l3 = shl_in(o.v[1]), r5 = shr_in(o.v[1]);
      if (hl) {
        l3 = e0[k];
        l1 = e1[k];
      }
      if (hr) r5 = e0[k];
      rs0[k] = h * o.v[0] + w1 * (l1 + o.v[1]) + w3 * (l3 + o.v[3]);
      rs1[k] = h * o.v[2] + w1 * (o.v[1] + o.v[3]) + w3 * (l1 + r5);
    }
#pragma unroll
    for (int s = 0; s < kCR; ++s) {
      const int J = J0 + s;
      if (J > Jl) break;
      const int m = 2 * s + 3;  // index of fine row 2J
      Vec<T, 2> out;
      out.v[0] = h * rs0[m] + w1 * (rs0[m - 1] + rs0[m + 1]) + w3 * (rs0[m - 3] + rs0[m + 3]);
      out.v[1] = h * rs1[m] + w1 * (rs1[m - 1] + rs1[m + 1]) + w3 * (rs1[m - 3] + rs1[m + 3]);
      *reinterpret_cast<Vec<T, 2>*>(coarse + (int64_t)J * nc + c / 2) = out;
    }
  }
}

// fine += P coarse.  For coarse row J the lane forms the x-interpolated
// values at its four fine columns,
//   tx(J) = (e(I0), (-e(I0-1) + 9 e(I0) + 9 e(I1) - e(I1+1)) / 16,
//            e(I1), (-e(I0) + 9 e(I1) + 9 e(I1+1) - e(I1+2)) / 16),
// then fine row 2J = tx(J) and 2J+1 = (-tx(J-1) + 9 tx(J) + 9 tx(J+1) - tx(J+2)) / 16.
template <typename T>
__global__ void __launch_bounds__(kTPB) k_prolong_tile(TArgs A, const T* __restrict__ coarse,
                                                       T* __restrict__ fine) {
  constexpr int NC = kCR + 3;
  const int nf = A.nf, nc = A.nc, cmask = nc - 1;
  const int lane = threadIdx.x & 63;
  const bool hl = lane == 0, hr = lane == 63;
  const T k9 = T(9), k16 = T(0.0625);
  const int inst = blockIdx.x / A.bpi;
  coarse += (int64_t)inst * A.sc;
  fine += (int64_t)inst * A.sf;
  for (int t = (blockIdx.x - inst * A.bpi) * (kTPB / 64) + (threadIdx.x >> 6); t < A.tiles;
       t += A.bpi * (kTPB / 64)) {
    const int rg = t / A.wstrips;
    const int strip = t - rg * A.wstrips;
    const int J0 = rg * kCR;
    const int Jl = min(J0 + kCR, nc + 1) - 1;
    const int c = strip * 256 + 4 * lane;  // fine columns c .. c+3
    const int I0 = c / 2;
    const int hcol = hl ? ((I0 - 2) & cmask) : ((I0 + 2) & cmask);
    // every load of the tile first (their latencies overlap): the coarse rows
    // J0-1 .. Jl+2 (reflected; rows a short last tile does not reach repeat
    // row Jl+2 and are unused), the halo columns of lanes 0 and 63 (lane 0:
    // I0-2, I0-1; lane 63: I1+1, I1+2), and the fine rows the tile updates
    // (clamped to valid rows; rows past the tile are not stored)
    Vec<T, 2> eo[NC];
    T g0[NC], g1[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T* row = coarse + (int64_t)refl(min(J0 - 1 + k, Jl + 2), nc) * nc;
      eo[k] = *reinterpret_cast<const Vec<T, 2>*>(row + I0);
      g0[k] = g1[k] = T(0);
    }
    if (hl || hr) {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const T* row = coarse + (int64_t)refl(min(J0 - 1 + k, Jl + 2), nc) * nc;
        const Vec<T, 2> hv = *reinterpret_cast<const Vec<T, 2>*>(row + hcol);
        g0[k] = hv.v[0];
        g1[k] = hv.v[1];
      }
    }
    Vec<T, 4> fv[2 * kCR];
#pragma unroll
    for (int r = 0; r < 2 * kCR; ++r)
      fv[r] = *reinterpret_cast<const Vec<T, 4>*>(fine + (int64_t)min(2 * J0 + r, nf) * nf + c);
    T tx[NC][4];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const Vec<T, 2>& e = eo[k];
      T em1 = shl_in(e.v[1]), ep2 = shr_in(e.v[0]), ep3 = shr_in(e.v[1]);
      if (hl) em1 = g1[k];
      if (hr) {
        ep2 = g0[k];
        ep3 = g1[k];
      }
      tx[k][0] = e.v[0];
      tx[k][1] = (-em1 + k9 * e.v[0] + k9 * e.v[1] - ep2) * k16;
      tx[k][2] = e.v[1];
      tx[k][3] = (-e.v[0] + k9 * e.v[1] + k9 * ep2 - ep3) * k16;
    }
#pragma unroll
    for (int s = 0; s < kCR; ++s) {
      const int J = J0 + s;
      if (J > Jl) break;
      const int k = s + 1;  // index of coarse row J
      {
        Vec<T, 4>* dst = reinterpret_cast<Vec<T, 4>*>(fine + (int64_t)(2 * J) * nf + c);
        Vec<T, 4> v = fv[2 * s];
#pragma unroll
        for (int i = 0; i < 4; ++i) v.v[i] += tx[k][i];
        *dst = v;
      }
      if (2 * J + 1 <= nf) {
        Vec<T, 4>* dst = reinterpret_cast<Vec<T, 4>*>(fine + (int64_t)(2 * J + 1) * nf + c);
        Vec<T, 4> v = fv[2 * s + 1];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          v.v[i] += (-tx[k - 1][i] + k9 * tx[k][i] + k9 * tx[k + 1][i] - tx[k + 2][i]) * k16;
        *dst = v;
      }
    }
  }
}

TArgs targs(int nf, int& blocks) {
  TArgs A;
  A.nf = nf;
  A.nc = nf / 2;
  A.wstrips = nf / 256;
  A.tiles = A.wstrips * ((A.nc + 1 + kCR - 1) / kCR);
  const BatchCtx& B = g_batch;
  const int count = B.count > 1 ? B.count : 1;
  const int cap = kMaxBlocks / count > 0 ? kMaxBlocks / count : 1;
  const int64_t b = ((int64_t)A.tiles + kTPB / 64 - 1) / (kTPB / 64);
  A.bpi = (int)(b < cap ? b : cap);
  A.sf = count > 1 ? B.stride : 0;
  A.sc = count > 1 ? B.stride_c : 0;
  blocks = A.bpi * count;
  return A;
}

}  // namespace

// Single fine grids from 2048 up use the tiled transfers; below, the
// one-node-per-thread kernels, whose many short threads finish sooner there
// (measured per launch, float32: nf = 1024 restriction 6.5 us against 8.4
// tiled, 512 and 256 about 4.7 against 7-8; nf = 2048 prolongation 21 us
// against 9.8 tiled).  BF_TRANSFER_TILE_MIN overrides the threshold (>= 256).
bool transfer_stream_ok(int nf) {
  static const int lim = [] {
    const char* v = std::getenv("BF_TRANSFER_TILE_MIN");
    const int x = v ? std::atoi(v) : 0;
    return x >= 256 ? x : 2048;
  }();
  return nf >= lim;
}

template <typename T>
void stream_prolong_add(int nf, const T* coarse, T* fine, hipStream_t st) {
  int blocks;
  const TArgs A = targs(nf, blocks);
  hipLaunchKernelGGL((k_prolong_tile<T>), dim3(blocks), dim3(kTPB), 0, st, A, coarse, fine);
}

template <typename T>
void stream_restrict(int nf, const T* fine, T* coarse, hipStream_t st) {
  int blocks;
  const TArgs A = targs(nf, blocks);
  hipLaunchKernelGGL((k_restrict_tile<T>), dim3(blocks), dim3(kTPB), 0, st, A, fine, coarse);
}

template void stream_prolong_add<double>(int, const double*, double*, hipStream_t);
template void stream_prolong_add<float>(int, const float*, float*, hipStream_t);
template void stream_restrict<double>(int, const double*, double*, hipStream_t);
template void stream_restrict<float>(int, const float*, float*, hipStream_t);

}  // namespace bf
