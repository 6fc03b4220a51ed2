// Streaming grid-transfer kernels for the large levels.
//
// Cubic interpolation P and its weighted adjoint R = 1/4 W_c^-1 P^T W_f
// (tensor products of the 1-D weights (-1, 9, 16, 9, -1)/16 and
// {0: 1/2, +-1: 9/32, +-3: -1/32}), periodic in x, even reflection in y.
//
// Both kernels give each lane one coarse column I (fine columns 2I, 2I+1)
// and walk a chunk of coarse rows, keeping a sliding window in registers so
// that every coarse or fine value is fetched from memory once per tile; the
// coarse neighbours I-1, I+1, I+2 (prolongation) and the fine neighbours
// 2I-3, 2I-1, 2I+3 (restriction) come from a one-row LDS exchange.  Tiles are
// dealt to XCDs in contiguous ranges (block b runs on XCD b % 8).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace bf {

template <typename T>
struct TransferArgs {
  Geo F, C;
  const T* in;
  T* out;
  int cy, chunks, tiles, per_xcd;
};

template <typename T>
struct alignas(2 * sizeof(T)) Two {
  T x, y;
};

// fine += P coarse.  Lane = coarse column I; the window holds, for coarse
// rows J-1 .. J+2, the x-interpolated values at the lane's fine columns:
// tx(J) = (e(J, I), (-e(J,I-1) + 9 e(J,I) + 9 e(J,I+1) - e(J,I+2)) / 16).
// Fine row 2J = tx(J); fine row 2J+1 = (-tx(J-1) + 9 tx(J) + 9 tx(J+1) - tx(J+2)) / 16.
template <int TPB, typename T>
__global__ void __launch_bounds__(TPB) k_prolong_stream(TransferArgs<T> P) {
  __shared__ T row[TPB + 3];
  const int bid = blockIdx.x;
  const int t = (bid & 7) * P.per_xcd + (bid >> 3);
  if (t >= P.tiles) return;
  const int nc = P.C.n, cmask = P.C.mask, nf = P.F.n;
  const int strip = t / P.chunks;
  const int chunk = t - strip * P.chunks;
  const int J0 = chunk * P.cy;
  const int J1 = min(J0 + P.cy, nc + 1);  // coarse rows J0 .. J1-1
  const int tid = threadIdx.x;
  const int I = strip * TPB + tid;
  const T* __restrict__ E = P.in;
  T* __restrict__ Fo = P.out;

  // x-interpolate coarse row JJ (reflected) for this lane: needs columns
  // I-1 .. I+2; the block loads columns strip*TPB - 1 .. strip*TPB + TPB + 1.
  auto tx_row = [&](int JJ) -> Two<T> {
    const T* er = E + (int64_t)refl(JJ, nc) * nc;
    const int base = strip * TPB;
    __syncthreads();  // previous readers of row[] are done
    row[tid + 1] = er[I];
    if (tid < 3) {
      const int col = tid == 0 ? (base - 1) & cmask : (base + TPB + tid - 1) & cmask;
      row[tid == 0 ? 0 : TPB + tid] = er[col];
    }
    __syncthreads();
    const T em1 = row[tid], e0 = row[tid + 1], e1 = row[tid + 2], e2 = row[tid + 3];
    return Two<T>{e0, (-em1 + T(9) * e0 + T(9) * e1 - e2) * T(0.0625)};
  };

  Two<T> w0 = tx_row(J0 - 1), w1 = tx_row(J0), w2 = tx_row(J0 + 1), w3 = tx_row(J0 + 2);
  for (int J = J0; J < J1; ++J) {
    // fine row 2J
    {
      Two<T>* dst = reinterpret_cast<Two<T>*>(Fo + (int64_t)(2 * J) * nf + 2 * I);
      Two<T> v = *dst;
      v.x += w1.x;
      v.y += w1.y;
      *dst = v;
    }
    if (2 * J + 1 <= nf) {
      Two<T>* dst = reinterpret_cast<Two<T>*>(Fo + (int64_t)(2 * J + 1) * nf + 2 * I);
      Two<T> v = *dst;
      v.x += (-w0.x + T(9) * w1.x + T(9) * w2.x - w3.x) * T(0.0625);
      v.y += (-w0.y + T(9) * w1.y + T(9) * w2.y - w3.y) * T(0.0625);
      *dst = v;
    }
    w0 = w1;
    w1 = w2;
    w2 = w3;
    if (J + 1 < J1) w3 = tx_row(J + 3);
  }
}

// coarse = R fine.  Lane = coarse column I; per fine row f the lane forms
// rs(f) = 1/2 r(f,2I) + 9/32 (r(f,2I-1) + r(f,2I+1)) - 1/32 (r(f,2I-3) + r(f,2I+3))
// and coarse(J, I) = 1/2 rs(2J) + 9/32 (rs(2J-1) + rs(2J+1)) - 1/32 (rs(2J-3) + rs(2J+3)),
// fine rows reflected.  The window keeps rs for fine rows 2J-3 .. 2J+3.
template <int TPB, typename T>
__global__ void __launch_bounds__(TPB) k_restrict_stream(TransferArgs<T> P) {
  __shared__ T row[2 * TPB + 8];
  const int bid = blockIdx.x;
  const int t = (bid & 7) * P.per_xcd + (bid >> 3);
  if (t >= P.tiles) return;
  const int nf = P.F.n, fmask = P.F.mask, nc = P.C.n;
  const int strip = t / P.chunks;
  const int chunk = t - strip * P.chunks;
  const int J0 = chunk * P.cy;
  const int J1 = min(J0 + P.cy, nc + 1);
  const int tid = threadIdx.x;
  const int I = strip * TPB + tid;
  const int base = 2 * strip * TPB;  // first fine column of the strip
  const T* __restrict__ Fi = P.in;

  // row[] holds fine columns base-4 .. base+2*TPB+3 at index (col - base + 4)
  auto rs_row = [&](int f) -> T {
    const T* fr = Fi + (int64_t)refl(f, nf) * nf;
    __syncthreads();
    *reinterpret_cast<Two<T>*>(&row[2 * tid + 4]) = *reinterpret_cast<const Two<T>*>(fr + 2 * I);
    if (tid < 8) {
      const int k = tid < 4 ? tid : 2 * TPB + tid;  // 0..3 | 2TPB+4 .. 2TPB+7
      row[k] = fr[(base - 4 + k) & fmask];
    }
    __syncthreads();
    const int k = 2 * tid + 4;
    return T(0.5) * row[k] + T(9.0 / 32) * (row[k - 1] + row[k + 1]) -
           T(1.0 / 32) * (row[k - 3] + row[k + 3]);
  };

  // window: r[m] = rs(2J - 3 + m), m = 0..6
  T r0 = rs_row(2 * J0 - 3), r1 = rs_row(2 * J0 - 2), r2 = rs_row(2 * J0 - 1);
  T r3 = rs_row(2 * J0), r4 = rs_row(2 * J0 + 1), r5 = rs_row(2 * J0 + 2);
  T r6 = rs_row(2 * J0 + 3);
  for (int J = J0; J < J1; ++J) {
    P.out[(int64_t)J * nc + I] =
        T(0.5) * r3 + T(9.0 / 32) * (r2 + r4) - T(1.0 / 32) * (r0 + r6);
    if (J + 1 < J1) {
      r0 = r2;
      r1 = r3;
      r2 = r4;
      r3 = r5;
      r4 = r6;
      r5 = rs_row(2 * J + 4);
      r6 = rs_row(2 * J + 5);
    }
  }
  (void)r1;
}

namespace {

struct TCfg {
  int tpb, cy, chunks, tiles, per_xcd, blocks;
};

TCfg transfer_cfg(int nc) {
  TCfg c;
  c.tpb = nc >= 256 ? 256 : (nc >= 128 ? 128 : 64);
  const int strips = nc / c.tpb;
  int cy = (int)(((int64_t)(nc + 1) * strips) / 2048);
  cy = cy < 4 ? 4 : (cy > 32 ? 32 : cy);
  c.cy = cy;
  c.chunks = (nc + 1 + cy - 1) / cy;
  c.tiles = strips * c.chunks;
  c.per_xcd = (c.tiles + 7) / 8;
  c.blocks = 8 * c.per_xcd;
  return c;
}

template <typename T>
TransferArgs<T> targs(int nf, const T* in, T* out, const TCfg& c) {
  TransferArgs<T> P;
  P.F = make_geo(nf);
  P.C = make_geo(nf / 2);
  P.in = in;
  P.out = out;
  P.cy = c.cy;
  P.chunks = c.chunks;
  P.tiles = c.tiles;
  P.per_xcd = c.per_xcd;
  return P;
}

}  // namespace

bool transfer_stream_ok(int nf) { return nf / 2 >= 64; }

template <typename T>
void stream_prolong_add(int nf, const T* coarse, T* fine, hipStream_t st) {
  const TCfg c = transfer_cfg(nf / 2);
  const TransferArgs<T> P = targs(nf, coarse, fine, c);
  if (c.tpb == 256)
    hipLaunchKernelGGL((k_prolong_stream<256, T>), dim3(c.blocks), dim3(256), 0, st, P);
  else if (c.tpb == 128)
    hipLaunchKernelGGL((k_prolong_stream<128, T>), dim3(c.blocks), dim3(128), 0, st, P);
  else
    hipLaunchKernelGGL((k_prolong_stream<64, T>), dim3(c.blocks), dim3(64), 0, st, P);
}

template <typename T>
void stream_restrict(int nf, const T* fine, T* coarse, hipStream_t st) {
  const TCfg c = transfer_cfg(nf / 2);
  const TransferArgs<T> P = targs(nf, fine, coarse, c);
  if (c.tpb == 256)
    hipLaunchKernelGGL((k_restrict_stream<256, T>), dim3(c.blocks), dim3(256), 0, st, P);
  else if (c.tpb == 128)
    hipLaunchKernelGGL((k_restrict_stream<128, T>), dim3(c.blocks), dim3(128), 0, st, P);
  else
    hipLaunchKernelGGL((k_restrict_stream<64, T>), dim3(c.blocks), dim3(64), 0, st, P);
}

template void stream_prolong_add<double>(int, const double*, double*, hipStream_t);
template void stream_prolong_add<float>(int, const float*, float*, hipStream_t);
template void stream_restrict<double>(int, const double*, double*, hipStream_t);
template void stream_restrict<float>(int, const float*, float*, hipStream_t);

}  // namespace bf
