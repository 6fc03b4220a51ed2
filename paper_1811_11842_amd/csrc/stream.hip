// Stencil kernels for the large grid levels.
//
// Tiling: every wavefront owns one tile of RPW output rows by 128 columns
// (two adjacent columns per lane: 16-byte loads and stores for float64, 8-byte
// for float32; four float32 columns per lane, 256 per wavefront, measured 4%
// slower on the float32 V-cycle of the 4096^2 step: half as many wavefronts,
// more registers each).  It issues all loads of the tile at once -- the RPW + 2R
// input rows of its columns (R = 1 for the 5-point and 2 for the 13-point
// operator; ghost rows are the reflected rows of the two-layer even
// reflection, paper Sec. 4, eq. discreteBC) and the epilogue's other inputs
// -- and takes the horizontal neighbours of each value from the adjacent
// lanes with DPP wave shifts; lanes 0 and 63 load the two columns beyond the
// wavefront's edge (periodic wrap) themselves.  No LDS and no barriers: each
// wavefront works on its own, and there are many short ones.
//
// Launch order: tiles are numbered row-group-major (all column strips of rows
// j0 .. j0+RPW-1, then the next row group) and handed to consecutive
// wavefronts, and the hardware deals consecutive workgroups round-robin to
// the 8 XCDs.  The wavefronts resident at any moment therefore cover one
// compact band of rows, which streams through DRAM like a copy; the input
// rows shared by neighbouring tiles (2R per tile) are read by neighbouring
// wavefronts at about the same time and mostly hit in cache.  (Dealing
// contiguous tile ranges to each XCD, or walking long chunks of rows per
// workgroup with a register window, measured 10-20% slower on 4096^2.)
// Outputs are stored non-temporally.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "stencil_ops.hpp"

namespace bf {

enum Epi {
  E_APPLY = 0,         // out = A x
  E_APPLY_DOT = 1,     // out = A x, partials of <x, A x>_W
  E_RESID = 2,         // out = b - A x
  E_RESID_NORM = 3,    // out = b - A x, partials of ||out||_W^2
  E_SMOOTH = 4,        // out = x + a D^{-1}(b - A x) + g (x - xprev)
  E_APPLY_DOT_DD = 5,  // out = A x (double-double), partials of <x, A x>_W
  E_RESID_DD = 6,      // out = b - A x (double-double), partials of ||out||^2 and sum ulp(x)^2
  E_SMOOTH_XB = 7,     // E_SMOOTH with x = a0 D^{-1} b formed on load (first sweep from 0
                       // folded into the second), xprev = 0
  E_SMOOTH_PB = 8,     // E_SMOOTH with xprev = a0 D^{-1} b formed on the fly
  E_SMOOTH_DOT = 9,    // E_SMOOTH and partials of <b, out>_W
  E_CG_P = 10,         // CG step: p' = z + beta p formed on load; out = A p' (double-double
                       // for the CH operator), out2 = p', partials of <p', A p'>_W, and the
                       // deferred x += alpha p (alpha, beta from device scalars)
  E_SMOOTH_DOT2 = 11,  // E_SMOOTH and partials of <b, out>_W and <out, q>_W (q float64)
  E_CG_P32 = 12,       // E_CG_P with z read from a float32 field (z32): the float32
                       // V-cycle's output, stored at the precision it has
  E_GUESS = 13         // no output: partials of <b, A x>_W, <A x, A x>_W and <b, b>_W
                       // (the least-squares initial guess and ||b|| in one pass)
};

constexpr int kStreamTPB = 256;         // 4 wavefronts per workgroup
constexpr int kLaneCols = 2;            // columns per lane

// Vector of V elements of T (one load or store).
template <typename T, int V>
struct alignas(sizeof(T) * V) VecN {
  T v[V];
};

template <typename T, typename TO>
struct StreamArgs {
  OpDesc A;
  Geo G;
  const T* x;
  const T* b;
  const T* xprev;
  TO* out;
  double* partials;
  double a, g, a0;
  int rgroups;         // row groups of RPW rows
  int wstrips;         // column strips of 128 columns
  int tiles;           // rgroups * wstrips
  double* out2;        // E_CG_P: p'
  double* xu;          // E_CG_P: x (updated in place; null: x is not updated)
  const double* scal;  // E_CG_P: device scalars (alpha, beta)
  const double* q;     // E_SMOOTH_DOT2: second vector of the extra dot
  int first;           // E_CG_P: first step after a (re)start: p' = z, no x update
  const float* z32;    // E_CG_P32: z
  const float* p32_old;  // E_CG_P32: p_old (float32)
  float* p32_new;        // E_CG_P32: p' rounded to float32
  float* out32;        // E_RESID_DD (optional): float32 copy of out
  // Batch of equal-sized instances stored bstride elements apart: workgroups
  // bpi * i .. bpi * (i+1) - 1 work on instance i (their partials are the
  // instance's), device scalars are kNumSlots apart.  bcoef (optional): per
  // instance kCoefStride doubles {coef, dinv_int, dinv_edge, a[8], g[8]}
  // replacing A's coefficients and a = a[ia], g = g[ig], a0 = a[ia0].
  // active (optional): instances with active[i] == 0 are skipped.
  int batch, bpi;
  int64_t bstride;
  const double* bcoef;
  int ia, ig, ia0;
  const int* active;
};

// Lane i receives the value of lane i-1 (DPP wave_shr:1) or of lane i+1
// (wave_shl:1).  The lane without a source (lane 0, resp. lane 63) keeps
// `edge` -- the DPP's old value -- which is where the caller puts the halo
// column that lane loaded itself, so no select follows the shift.
__device__ __forceinline__ float from_left(float v, float edge) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138,
                                                    0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v, float edge) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130,
                                                    0xf, 0xf, false));
}
__device__ __forceinline__ double from_left(double v, double edge) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(edge), __double2loint(v), 0x138, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(edge), __double2hiint(v), 0x138, 0xf,
                                             0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v, double edge) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(edge), __double2loint(v), 0x130, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(edge), __double2hiint(v), 0x130, 0xf,
                                             0xf, false);
  return __hiloint2double(hi, lo);
}

// Largest value over the 64 lanes of a wavefront, returned in a scalar
// register: an inclusive max-scan within each 16-lane row by DPP row shifts
// (1, 2, 4, 8; lanes without a source take 0, the identity of unsigned max),
// then the row maxima carried across rows by DPP row broadcasts (lane 15 into
// rows 1 and 3, lane 31 into rows 2 and 3); lane 63 ends with the maximum.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  auto dpp = [](uint32_t x, int ctrl, int row_mask) -> uint32_t {
    switch (ctrl) {  // the DPP control must be a constant
      case 0x111: return __builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
      case 0x112: return __builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
      case 0x114: return __builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
      case 0x118: return __builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
      case 0x142: return __builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
      default: return __builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
    }
    (void)row_mask;
  };
  v = max(v, dpp(v, 0x111, 0xf));  // row_shr:1
  v = max(v, dpp(v, 0x112, 0xf));  // row_shr:2
  v = max(v, dpp(v, 0x114, 0xf));  // row_shr:4
  v = max(v, dpp(v, 0x118, 0xf));  // row_shr:8
  v = max(v, dpp(v, 0x142, 0xa));  // row_bcast:15
  v = max(v, dpp(v, 0x143, 0xc));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// One input row of a lane: its V values and, on lanes 0 and 63, the two
// values beyond the wavefront's edge (lane 0: columns c-2, c-1; lane 63:
// columns c+V, c+V+1).
template <typename T, int V>
struct XRow {
  T o[V];
  T h0, h1;
};

// Non-temporal store of a vector (the outputs are not re-read by this kernel).
template <typename T, int V>
__device__ __forceinline__ void store_nt(VecN<T, V>* dst, const VecN<T, V>& v) {
#pragma unroll
  for (int i = 0; i < V; ++i) __builtin_nontemporal_store(v.v[i], &dst->v[i]);
}

template <int OP, int EPI, int RPW, typename T, typename TO>
__global__ void __launch_bounds__(kStreamTPB) k_stream(StreamArgs<T, TO> P) {
  constexpr int V = kLaneCols;
  constexpr int R = (OP == 1) ? 2 : 1;
  constexpr int NR = RPW + 2 * R;
  constexpr bool SMOOTH = (EPI == E_SMOOTH || EPI == E_SMOOTH_XB || EPI == E_SMOOTH_PB ||
                           EPI == E_SMOOTH_DOT || EPI == E_SMOOTH_DOT2);
  constexpr bool RED = (EPI == E_APPLY_DOT || EPI == E_RESID_NORM || EPI == E_APPLY_DOT_DD ||
                        EPI == E_RESID_DD || EPI == E_SMOOTH_DOT || EPI == E_CG_P ||
                        EPI == E_CG_P32 || EPI == E_GUESS ||
                        EPI == E_SMOOTH_DOT2);
  constexpr bool RED2 = (EPI == E_RESID_DD || EPI == E_SMOOTH_DOT2 || EPI == E_GUESS);
  constexpr bool RED3 = EPI == E_GUESS;
  constexpr bool NEEDB = (EPI == E_RESID || EPI == E_RESID_NORM || SMOOTH || EPI == E_RESID_DD ||
                          EPI == E_GUESS);
  constexpr bool NEEDP = (EPI == E_SMOOTH || EPI == E_SMOOTH_DOT || EPI == E_SMOOTH_DOT2);
  using VT = VecN<T, V>;
  using VO = VecN<TO, V>;

  const int n = P.G.n, mask = P.G.mask;
  const int lane = threadIdx.x & 63;
  const bool hl = lane == 0, hr = lane == 63;
  const int inst = blockIdx.x / P.bpi;
  const int lblock = blockIdx.x - inst * P.bpi;
  const int64_t ioff = (int64_t)inst * P.bstride;
  const T* const Xp = P.x + ioff;
  const T* const Bp = P.b ? P.b + ioff : nullptr;
  const T* const XPp = P.xprev ? P.xprev + ioff : nullptr;
  TO* const Op = P.out + ioff;
  double* const O2p = P.out2 ? P.out2 + ioff : nullptr;
  double* const XUp = P.xu ? P.xu + ioff : nullptr;
  const double* const Qp = P.q ? P.q + ioff : nullptr;
  double cf = P.A.coef, di = P.A.dinv_int, de = P.A.dinv_edge;
  double pa = P.a, pg = P.g, pa0 = P.a0;
  if (P.bcoef) {
    const double* rc = P.bcoef + (int64_t)inst * kCoefStride;
    cf = rc[0];
    di = rc[1];
    de = rc[2];
    pa = rc[3 + P.ia];
    pg = rc[11 + P.ig];
    pa0 = rc[3 + P.ia0];
  }
  const T ca = T(pa), cg = T(pg), ca0 = T(pa0);
  double beta = 0.0, alpha_prev = 0.0;
  constexpr bool CGP = (EPI == E_CG_P || EPI == E_CG_P32);
  if constexpr (CGP) {
    if (!P.first) {
      beta = P.scal[(int64_t)inst * kNumSlots + S_BETA];
      alpha_prev = P.scal[(int64_t)inst * kNumSlots + S_ALPHA];
    }
  }
  const T tdi = T(di), tde = T(de), tcoef = T(cf);
  auto dinv_row = [&](int jr) -> T { return row_dinv<OP, T>(tdi, tde, jr, n); };
  double acc = 0.0, acc2 = 0.0, acc3 = 0.0;
  const bool skip = P.active && !P.active[inst];

  const int wpb = kStreamTPB / 64;
  // the tile index is the same on every lane of a wavefront: keeping it in a
  // scalar register makes the row arithmetic (reflection, row addresses,
  // bounds) scalar
  const int t0 = __builtin_amdgcn_readfirstlane(lblock * wpb + (threadIdx.x >> 6));
  for (int t = t0; !skip && t < P.tiles; t += P.bpi * wpb) {
    const int rg = t / P.wstrips;
    const int strip = t - rg * P.wstrips;
    const int j0 = rg * RPW;
    const int jl = min(j0 + RPW, n + 1) - 1;  // last output row of the tile
    const int c = strip * (64 * V) + V * lane;
    const int hcol = hl ? ((c - V) & mask) : ((c + V) & mask);

    // Every load of the tile is issued before any value is used, so that
    // their latencies overlap (a load followed by its use in the same loop
    // iteration makes the wavefront wait for each row in turn): the window
    // rows j0-R .. jl+R (reflected; the rows a short last tile does not reach
    // repeat row jl+R: they are no output's neighbour and leave the window's
    // largest magnitude unchanged), then the halo columns of lanes 0 and 63
    // (rows 1 .. NR-2 of the window, the centre or vertical neighbours of an
    // output, in one lane-divergent block), then the epilogue's inputs at the
    // output rows (clamped to the last row; rows past it are not stored).
    int jrw[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) jrw[k] = refl(min(j0 - R + k, jl + R), n);
    const bool cg_beta = CGP && !P.first;
    XRow<T, V> xr[NR];
    XRow<T, V> po[CGP ? NR : 1];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if constexpr (EPI == E_CG_P32) {
        // z in float32 (8 bytes per lane), widened to T
        const float2 zv = *reinterpret_cast<const float2*>(P.z32 + ioff + (int64_t)jrw[k] * n + c);
        xr[k].o[0] = T(zv.x);
        xr[k].o[1] = T(zv.y);
      } else {
        const VT v = *reinterpret_cast<const VT*>(Xp + (int64_t)jrw[k] * n + c);
#pragma unroll
        for (int i = 0; i < V; ++i) xr[k].o[i] = v.v[i];
      }
      xr[k].h0 = xr[k].h1 = T(0);
    }
    if constexpr (CGP) {
      if (cg_beta) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          if constexpr (EPI == E_CG_P32) {
            const float2 v =
                *reinterpret_cast<const float2*>(P.p32_old + ioff + (int64_t)jrw[k] * n + c);
            po[k].o[0] = T(v.x);
            po[k].o[1] = T(v.y);
          } else {
            const VT v = *reinterpret_cast<const VT*>(XPp + (int64_t)jrw[k] * n + c);
#pragma unroll
            for (int i = 0; i < V; ++i) po[k].o[i] = v.v[i];
          }
          po[k].h0 = po[k].h1 = T(0);
        }
      }
    }
    // lane 0 holds columns c-2, c-1 and lane 63 columns c+2, c+3 in h0, h1
    if (hl || hr) {
#pragma unroll
      for (int k = 1; k < NR - 1; ++k) {
        if constexpr (EPI == E_CG_P32) {
          const float2 zh =
              *reinterpret_cast<const float2*>(P.z32 + ioff + (int64_t)jrw[k] * n + hcol);
          xr[k].h0 = T(zh.x);
          xr[k].h1 = T(zh.y);
        } else {
          const VT h = *reinterpret_cast<const VT*>(Xp + (int64_t)jrw[k] * n + hcol);
          xr[k].h0 = h.v[0];
          xr[k].h1 = h.v[1];
        }
        if constexpr (EPI == E_CG_P32) {
          if (cg_beta) {
            const float2 h =
                *reinterpret_cast<const float2*>(P.p32_old + ioff + (int64_t)jrw[k] * n + hcol);
            po[k].h0 = T(h.x);
            po[k].h1 = T(h.y);
          }
        } else if constexpr (CGP) {
          if (cg_beta) {
            const VT h = *reinterpret_cast<const VT*>(XPp + (int64_t)jrw[k] * n + hcol);
            po[k].h0 = h.v[0];
            po[k].h1 = h.v[1];
          }
        }
      }
    }
    constexpr bool DOT2Q = EPI == E_SMOOTH_DOT2;
    VT bo[NEEDB ? RPW : 1], pco[NEEDP ? RPW : 1] = {};
    VecN<double, V> qo[DOT2Q ? RPW : 1], xo[CGP ? RPW : 1];
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int64_t o = (int64_t)min(j0 + s, jl) * n + c;
      if constexpr (NEEDB) bo[s] = *reinterpret_cast<const VT*>(Bp + o);
      if constexpr (DOT2Q) qo[s] = *reinterpret_cast<const VecN<double, V>*>(Qp + o);
    }
    if constexpr (NEEDP) {
      if (XPp) {
#pragma unroll
        for (int s = 0; s < RPW; ++s)
          pco[s] = *reinterpret_cast<const VT*>(XPp + (int64_t)min(j0 + s, jl) * n + c);
      }
    }
    if constexpr (CGP) {
      if (cg_beta && XUp) {
#pragma unroll
        for (int s = 0; s < RPW; ++s)
          xo[s] = *reinterpret_cast<const VecN<double, V>*>(XUp + (int64_t)min(j0 + s, jl) * n + c);
      }
    }
    // p' = z + beta p_old (CG step); x1 = a0 D^{-1} b (first sweep from zero)
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if constexpr (CGP) {
        if (cg_beta) {
#pragma unroll
          for (int i = 0; i < V; ++i) xr[k].o[i] += beta * po[k].o[i];
          xr[k].h0 += beta * po[k].h0;
          xr[k].h1 += beta * po[k].h1;
        }
        if constexpr (EPI == E_CG_P32) {
          // the float32 search direction: q, <p', q> and x use the rounded p'
#pragma unroll
          for (int i = 0; i < V; ++i) xr[k].o[i] = T(float(xr[k].o[i]));
          xr[k].h0 = T(float(xr[k].h0));
          xr[k].h1 = T(float(xr[k].h1));
        }
      }
      if constexpr (EPI == E_SMOOTH_XB) {
        const T sc = ca0 * dinv_row(jrw[k]);
#pragma unroll
        for (int i = 0; i < V; ++i) xr[k].o[i] *= sc;
        xr[k].h0 *= sc;
        xr[k].h1 *= sc;
      }
    }

    // Cahn-Hilliard CG step: q = A p' exactly rounded through the split of
    // every window value against sigma = 2^7 times a power of two above the
    // largest |p'| of the wavefront's window (apply13_split); xr keeps the hi
    // parts, xl the lo parts.  The largest magnitude is found from the high
    // words (their unsigned order is the order of |value| for finite values).
    constexpr bool SPLIT = CGP && OP == 1 && std::is_same<T, double>::value;
    XRow<T, V> xl[SPLIT ? NR : 1];
    if constexpr (SPLIT) {
      uint32_t mx = 0;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
#pragma unroll
        for (int i = 0; i < V; ++i)
          mx = max(mx, (uint32_t)__double2hiint(xr[k].o[i]) & 0x7fffffffu);
        mx = max(mx, (uint32_t)__double2hiint(xr[k].h0) & 0x7fffffffu);
        mx = max(mx, (uint32_t)__double2hiint(xr[k].h1) & 0x7fffffffu);
      }
      // biased exponent eb: every |value| < 2^(eb - 1022); sigma = 2^(eb - 1015)
      const int eb = (int)(wave_max_u32(mx) >> 20);
      const double sigma = __hiloint2double(min(eb + 8, 2046) << 20, 0);
#pragma unroll
      for (int k = 0; k < NR; ++k) {
#pragma unroll
        for (int i = 0; i < V; ++i) split_sigma(xr[k].o[i], sigma, xr[k].o[i], xl[k].o[i]);
        split_sigma(xr[k].h0, sigma, xr[k].h0, xl[k].h0);
        split_sigma(xr[k].h1, sigma, xr[k].h1, xl[k].h1);
      }
    }

    // neighbours across lanes: column c-1, c-2 (left) and c+V, c+V+1 (right)
    // (lane 0 holds columns c-2, c-1 in h0, h1; lane 63 columns c+V, c+V+1)
    auto left1 = [&](const XRow<T, V>& r) { return from_left(r.o[V - 1], r.h1); };
    auto left2 = [&](const XRow<T, V>& r) { return from_left(r.o[V - 2], r.h0); };
    auto right1 = [&](const XRow<T, V>& r) { return from_right(r.o[0], r.h0); };
    auto right2 = [&](const XRow<T, V>& r) { return from_right(r.o[1], r.h1); };

    // the 5 (OP 0, 2) or 13 (OP 1) values around the lane's V nodes of window row k
    auto gather_nb = [&](const XRow<T, V>* W, int k, Nb13T<T>(&nb)[V]) {
      const XRow<T, V>& C = W[k];
      // centre row, columns c-2 .. c+V+1
      T e[V + 4];
      e[1] = left1(C);
      e[V + 2] = right1(C);
      if (OP == 1) {
        e[0] = left2(C);
        e[V + 3] = right2(C);
      } else {
        e[0] = e[V + 3] = T(0);
      }
#pragma unroll
      for (int i = 0; i < V; ++i) e[2 + i] = C.o[i];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        nb[i].c = e[i + 2];
        nb[i].xm1 = e[i + 1];
        nb[i].xp1 = e[i + 3];
        nb[i].ym1 = W[k - 1].o[i];
        nb[i].yp1 = W[k + 1].o[i];
      }
      if constexpr (OP == 1) {
        const XRow<T, V>& Mr = W[k - 1];
        const XRow<T, V>& Pr = W[k + 1];
        T m[V + 2], p[V + 2];  // rows j-1, j+1, columns c-1 .. c+V
        m[0] = left1(Mr);
        m[V + 1] = right1(Mr);
        p[0] = left1(Pr);
        p[V + 1] = right1(Pr);
#pragma unroll
        for (int i = 0; i < V; ++i) {
          m[1 + i] = Mr.o[i];
          p[1 + i] = Pr.o[i];
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
          nb[i].xm2 = e[i];
          nb[i].xp2 = e[i + 4];
          nb[i].ym2 = W[k - 2].o[i];
          nb[i].yp2 = W[k + 2].o[i];
          nb[i].dmm = m[i];
          nb[i].dmp = m[i + 2];
          nb[i].dpm = p[i];
          nb[i].dpp = p[i + 2];
        }
      }
    };

#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int j = j0 + s;
      if (j > jl) break;
      const int k = s + R;
      Nb13T<T> nb[V];
      gather_nb(xr, k, nb);
      const int64_t o = (int64_t)j * n + c;
      const double wgt = row_weight(j, n);
      const double cfj = row_coef<OP>(cf, j, n);
      const T coefj = (OP == 2 && (j == 0 || j == n)) ? T(0) : tcoef;
      VT bcur{}, pcur{};
      if constexpr (NEEDB) bcur = bo[s];
      if constexpr (NEEDP) pcur = pco[s];
      VO res;
      if constexpr (EPI == E_APPLY || EPI == E_APPLY_DOT) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
          const T ax = apply_vals<OP>(nb[i], coefj);
          res.v[i] = TO(ax);
          if (EPI == E_APPLY_DOT) acc += wgt * double(nb[i].c) * double(ax);
        }
      } else if constexpr (EPI == E_GUESS) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
          const double ax = double(apply_vals<OP>(nb[i], coefj));
          const double bv = double(bcur.v[i]);
          acc += wgt * bv * ax;
          acc2 += wgt * ax * ax;
          acc3 += wgt * bv * bv;
        }
      } else if constexpr (EPI == E_RESID || EPI == E_RESID_NORM) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
          const T r = bcur.v[i] - apply_vals<OP>(nb[i], coefj);
          res.v[i] = TO(r);
          if (EPI == E_RESID_NORM) acc += wgt * double(r) * double(r);
        }
      } else if constexpr (SMOOTH) {
        const T ad = ca * dinv_row(j);
        const T d0 = ca0 * dinv_row(j);
#pragma unroll
        for (int i = 0; i < V; ++i) {
          T prev = T(0);
          if (EPI == E_SMOOTH_PB)
            prev = d0 * bcur.v[i];
          else if (EPI != E_SMOOTH_XB && XPp)
            prev = pcur.v[i];
          const T xn =
              nb[i].c + ad * (bcur.v[i] - apply_vals<OP>(nb[i], coefj)) + cg * (nb[i].c - prev);
          res.v[i] = TO(xn);
          if (EPI == E_SMOOTH_DOT || EPI == E_SMOOTH_DOT2)
            acc += wgt * double(bcur.v[i]) * double(TO(xn));
        }
        if constexpr (EPI == E_SMOOTH_DOT2) {
#pragma unroll
          for (int i = 0; i < V; ++i) acc2 += wgt * double(res.v[i]) * qo[s].v[i];
        }
      } else if constexpr (std::is_same<T, double>::value) {
        if constexpr (EPI == E_APPLY_DOT_DD) {
#pragma unroll
          for (int i = 0; i < V; ++i) {
            res.v[i] = -residual_dd_vals<OP>(nb[i], 0.0, cfj);
            acc += wgt * nb[i].c * res.v[i];
          }
        } else if constexpr (CGP) {
          VecN<double, V> pn;
          if constexpr (SPLIT) {
            Nb13T<T> nbl[V];
            gather_nb(xl, k, nbl);
#pragma unroll
            for (int i = 0; i < V; ++i) {
              const double cv = nb[i].c + nbl[i].c;  // p' (exact: hi + lo)
              res.v[i] = apply13_split(nb[i], nbl[i], cv, cfj);
              acc += wgt * cv * res.v[i];
              pn.v[i] = cv;
            }
          } else {
#pragma unroll
            for (int i = 0; i < V; ++i) {
              res.v[i] = apply_vals<OP>(nb[i], T(cfj));
              acc += wgt * nb[i].c * res.v[i];
              pn.v[i] = nb[i].c;
            }
          }
          if constexpr (EPI == E_CG_P32) {
            VecN<float, V> pf;
#pragma unroll
            for (int i = 0; i < V; ++i) pf.v[i] = float(pn.v[i]);  // exact
            store_nt(reinterpret_cast<VecN<float, V>*>(P.p32_new + ioff + o), pf);
          } else {
            store_nt(reinterpret_cast<VecN<double, V>*>(O2p + o), pn);
          }
          if (cg_beta && XUp) {
            // the deferred x += alpha_prev p_old (p_old of this row: window row k)
            VecN<double, V> xv = xo[s];
#pragma unroll
            for (int i = 0; i < V; ++i) xv.v[i] += alpha_prev * double(po[k].o[i]);
            store_nt(reinterpret_cast<VecN<double, V>*>(XUp + o), xv);
          }
        } else if constexpr (EPI == E_RESID_DD) {
#pragma unroll
          for (int i = 0; i < V; ++i) {
            res.v[i] = residual_dd_vals<OP>(nb[i], bcur.v[i], cfj);
            acc += wgt * res.v[i] * res.v[i];
            const double u = ulp_of(nb[i].c);
            acc2 += wgt * u * u;
          }
          if (P.out32) {
            VecN<float, V> r32;
#pragma unroll
            for (int i = 0; i < V; ++i) r32.v[i] = float(res.v[i]);
            store_nt(reinterpret_cast<VecN<float, V>*>(P.out32 + ioff + o), r32);
          }
        }
      }
      if constexpr (EPI != E_GUESS) store_nt(reinterpret_cast<VO*>(Op + o), res);
    }
  }
  if constexpr (RED) {
    const double s1 = block_sum_n<kStreamTPB>(acc);
    if (threadIdx.x == 0) P.partials[blockIdx.x] = s1;
    if constexpr (RED2) {
      const double s2 = block_sum_n<kStreamTPB>(acc2);
      if (threadIdx.x == 0) P.partials[gridDim.x + blockIdx.x] = s2;
    }
    if constexpr (RED3) {
      const double s3 = block_sum_n<kStreamTPB>(acc3);
      if (threadIdx.x == 0) P.partials[2 * gridDim.x + blockIdx.x] = s3;
    }
  }
}

// Tile t of the overlapping-strip smoother passes (k_smooth3, k_smooth3r,
// k_smooth2, k_post): the four wavefronts of a workgroup take four
// consecutive row groups of one column strip (t = 4 q + w: strip q mod
// wstrips, row group 4 (q div wstrips) + w), so three of every four vertical
// tile boundaries -- whose halo rows both tiles load -- lie inside one
// workgroup and its CU's caches.  (With one row group per workgroup, the
// vertical neighbour of a tile is wstrips / 4 workgroups away, which the
// hardware's round-robin over the 8 XCDs puts on another XCD unless wstrips
// is a multiple of 32; these kernels have 34 to 38 strips at 4096^2: the
// grouped order lowered the fetched bytes of k_post and k_smooth3r by 16% and
// 25%, their times are unchanged, since they are bound by their arithmetic.)
// Tiles past the last row group are padding: the function returns false.
constexpr int kTileGroup = kStreamTPB / 64;

__device__ __forceinline__ bool grouped_tile(int t, int wstrips, int rgroups, int& rg,
                                             int& strip) {
  const int q = t / kTileGroup, w = t - q * kTileGroup;
  const int rb = q / wstrips;
  strip = q - rb * wstrips;
  rg = kTileGroup * rb + w;
  return rg < rgroups;
}

// Tile count of those kernels (padded to whole groups of row groups).
__host__ __device__ inline int grouped_tiles(int wstrips, int rgroups) {
  return wstrips * kTileGroup * ((rgroups + kTileGroup - 1) / kTileGroup);
}

// The Cahn-Hilliard CG step of a single grid (E_CG_P / E_CG_P32 for OP 1):
//   p' = z + beta p_old (p' = z on the first step), q = A p' = p' + s S13 p'
//   exactly rounded (apply13_split), partials of <p', q>_W, and the deferred
//   x += alpha_prev p_old.
// The wavefronts overlap by one lane on each side: a wavefront loads 128
// columns (two per lane) and lanes 1 .. 62 produce output (124 columns,
// strips 124 apart, the last one cut at n), so no lane loads halo columns
// and the split window holds only the lanes' own values (the register count
// decides the occupancy of this VALU-heavy kernel).  The DPP shifts bring the
// neighbours' columns; what lanes 0 and 63 receive from outside the
// wavefront only reaches their own discarded results.
constexpr int kCgLanes = 62;
constexpr int kCgCols = 2 * kCgLanes;

// p_old, p_new: the search directions, in the type of z (a float32 p' is
// p' = z + beta p_old rounded to float32; q, the reduction and the x update
// use the rounded value).
template <typename ZT>
struct CgArgs {
  OpDesc A;
  Geo G;
  const ZT* z;
  const ZT* p_old;
  ZT* p_new;
  double* q;
  double* x;  // null: no deferred x update (the caller updates x in batches)
  const double* scal;
  double* partials;
  int first;
  int rgroups, wstrips, tiles;
};

template <int RPW, typename ZT, int WAVES, bool FIRST, bool XU>
__global__ void __launch_bounds__(kStreamTPB) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
k_cg_ch(CgArgs<ZT> P) {
  constexpr int NR = RPW + 4;
  constexpr bool XUPD = !FIRST && XU;  // the deferred x += alpha_prev p_old
  const int n = P.G.n, mask = P.G.mask;
  const int lane = threadIdx.x & 63;
  double beta = 0.0, alpha_prev = 0.0;
  if (!FIRST) {
    beta = P.scal[S_BETA];
    alpha_prev = P.scal[S_ALPHA];
  }
  const double s13 = P.A.coef;
  double acc = 0.0;
  const int wpb = kStreamTPB / 64;
  const int t0 = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
  for (int t = t0; t < P.tiles; t += gridDim.x * wpb) {
    // one row group per wavefront, row-group-major (measured: the grouped
    // order of the smoother passes made this kernel 5% slower and raised its
    // fetched bytes)
    const int rg = t / P.wstrips;
    const int strip = t - rg * P.wstrips;
    const int j0 = rg * RPW;
    const int jl = min(j0 + RPW, n + 1) - 1;
    const int cu = strip * kCgCols + 2 * (lane - 1);  // unwrapped first column of the lane
    const int c = cu & mask;
    const bool out_lane = lane >= 1 && lane <= kCgLanes && cu < n;
    // Every load of the tile is issued before any value is used (no branch
    // between them), so their latencies overlap: the window rows j0-2 .. jl+2
    // (reflected; the rows a short last tile does not reach repeat row jl+2,
    // which leaves the window's largest magnitude unchanged and is never an
    // output's neighbour) of z and p_old, and x at the output rows.
    ZT zr[NR][2];
    double po[FIRST ? 1 : NR][2];
    double2 xo[XUPD ? RPW : 1];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int64_t ro = (int64_t)refl(min(j0 - 2 + k, jl + 2), n) * n + c;
      if constexpr (std::is_same<ZT, float>::value) {
        const float2 zv = *reinterpret_cast<const float2*>(P.z + ro);
        zr[k][0] = zv.x;
        zr[k][1] = zv.y;
      } else {
        const double2 zv = *reinterpret_cast<const double2*>(P.z + ro);
        zr[k][0] = zv.x;
        zr[k][1] = zv.y;
      }
      if constexpr (!FIRST) {
        if constexpr (std::is_same<ZT, float>::value) {
          const float2 pv = *reinterpret_cast<const float2*>(P.p_old + ro);
          po[k][0] = pv.x;
          po[k][1] = pv.y;
        } else {
          const double2 pv = *reinterpret_cast<const double2*>(P.p_old + ro);
          po[k][0] = pv.x;
          po[k][1] = pv.y;
        }
      }
    }
    if constexpr (XUPD) {
#pragma unroll
      for (int s = 0; s < RPW; ++s)
        xo[s] = *reinterpret_cast<const double2*>(P.x + (int64_t)min(j0 + s, jl) * n + c);
    }
    // p' = z + beta p_old over the window (rounded to the type of p)
    double w[NR][2];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        w[k][i] = zr[k][i];
        if constexpr (!FIRST) w[k][i] = double(ZT(w[k][i] + beta * po[k][i]));
      }
    }
    // the deferred x += alpha_prev p_old at the output rows (window rows 2 ..),
    // done first so that x and p_old leave the registers before the split
    if constexpr (XUPD) {
#pragma unroll
      for (int s = 0; s < RPW; ++s) {
        const int j = j0 + s;
        if (j > jl) break;
        if (out_lane) {
          double2 xv = xo[s];
          xv.x += alpha_prev * po[s + 2][0];
          xv.y += alpha_prev * po[s + 2][1];
          const int64_t o = (int64_t)j * n + c;
          __builtin_nontemporal_store(xv.x, P.x + o);
          __builtin_nontemporal_store(xv.y, P.x + o + 1);
        }
      }
    }
    // sigma: 2^7 times a power of two above every |p'| of the window
    uint32_t mx = 0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      mx = max(mx, (uint32_t)__double2hiint(w[k][0]) & 0x7fffffffu);
      mx = max(mx, (uint32_t)__double2hiint(w[k][1]) & 0x7fffffffu);
    }
    const int eb = (int)(wave_max_u32(mx) >> 20);
    const double sigma = __hiloint2double(min(eb + 8, 2046) << 20, 0);
    double wh[NR][2], wl[NR][2];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      split_sigma(w[k][0], sigma, wh[k][0], wl[k][0]);
      split_sigma(w[k][1], sigma, wh[k][1], wl[k][1]);
    }
    // the 13 values around the lane's two nodes (columns c, c+1) of window row k
    auto gather = [&](const double (*W)[2], int k, Nb13 (&nb)[2]) {
      const double l0 = from_left(W[k][0], 0.0), l1 = from_left(W[k][1], 0.0);
      const double r0 = from_right(W[k][0], 0.0), r1 = from_right(W[k][1], 0.0);
      const double ml1 = from_left(W[k - 1][1], 0.0), mr0 = from_right(W[k - 1][0], 0.0);
      const double pl1 = from_left(W[k + 1][1], 0.0), pr0 = from_right(W[k + 1][0], 0.0);
      // node c: columns c-2 = l0, c-1 = l1, c+1, c+2 = r0
      nb[0].c = W[k][0];
      nb[0].xm1 = l1;
      nb[0].xp1 = W[k][1];
      nb[0].xm2 = l0;
      nb[0].xp2 = r0;
      nb[0].ym1 = W[k - 1][0];
      nb[0].yp1 = W[k + 1][0];
      nb[0].ym2 = W[k - 2][0];
      nb[0].yp2 = W[k + 2][0];
      nb[0].dmm = ml1;
      nb[0].dmp = W[k - 1][1];
      nb[0].dpm = pl1;
      nb[0].dpp = W[k + 1][1];
      // node c+1: columns c-1 = l1, c, c+2 = r0, c+3 = r1
      nb[1].c = W[k][1];
      nb[1].xm1 = W[k][0];
      nb[1].xp1 = r0;
      nb[1].xm2 = l1;
      nb[1].xp2 = r1;
      nb[1].ym1 = W[k - 1][1];
      nb[1].yp1 = W[k + 1][1];
      nb[1].ym2 = W[k - 2][1];
      nb[1].yp2 = W[k + 2][1];
      nb[1].dmm = W[k - 1][0];
      nb[1].dmp = mr0;
      nb[1].dpm = W[k + 1][0];
      nb[1].dpp = pr0;
    };
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int j = j0 + s;
      if (j > jl) break;
      const int k = s + 2;
      Nb13 nh[2], nl[2];
      gather(wh, k, nh);
      gather(wl, k, nl);
      const int64_t o = (int64_t)j * n + c;
      const double wgt = row_weight(j, n);
      double2 qv, pv;
      pv.x = nh[0].c + nl[0].c;
      pv.y = nh[1].c + nl[1].c;
      qv.x = apply13_split(nh[0], nl[0], pv.x, s13);
      qv.y = apply13_split(nh[1], nl[1], pv.y, s13);
      if (out_lane) {
        acc += wgt * (pv.x * qv.x + pv.y * qv.y);
        __builtin_nontemporal_store(ZT(pv.x), P.p_new + o);  // exact: pv is a ZT value
        __builtin_nontemporal_store(ZT(pv.y), P.p_new + o + 1);
        __builtin_nontemporal_store(qv.x, P.q + o);
        __builtin_nontemporal_store(qv.y, P.q + o + 1);
      }
    }
  }
  const double s1 = block_sum_n<kStreamTPB>(acc);
  if (threadIdx.x == 0) P.partials[blockIdx.x] = s1;
}

// Three sweeps of the smoother from a zero iterate in one pass:
//   x1 = a0 D^{-1} b,  x2 = x1 + a1 D^{-1}(b - A x1) + g1 x1,
//   x3 = x2 + a2 D^{-1}(b - A x2) + g2 (x2 - x1).
// x1 is pointwise in b and x2 is formed in registers over the tile's rows
// widened by the stencil's reach, so the pass reads b and writes x3 only
// (the two-pass form also writes and re-reads x2).  x2 at a column needs x1
// two columns either side, and x3 needs x2 two columns either side, so the
// wavefronts overlap: each loads 128 columns (two per lane) but only lanes
// 2 .. 61 produce x3 (120 columns per wavefront, strips 120 columns apart,
// wrapped); the neighbours across lanes come from DPP shifts, and the values
// the edge lanes receive from outside the wavefront (zero) only reach lanes
// whose results are discarded.  Rows beyond the walls are the reflected rows;
// a stage-two value on a ghost row equals the one on its mirror row because
// the stencils are symmetric in y and every row coefficient is taken at the
// reflected index.
constexpr int kS3Lanes = 60;            // output lanes per wavefront
constexpr int kS3Cols = 2 * kS3Lanes;   // output columns per wavefront

// Batches of equal-sized instances for the fused passes (as for k_stream:
// workgroups bpi * i .. bpi * (i+1) - 1 work on instance i, fields bstride
// elements apart; with bcoef the coefficients and the smoother weights of
// sweeps k0, k0+1, k0+2 come from instance i's record; instances with
// active[i] == 0 are skipped).  Single grids: bpi = all workgroups.
struct FusedBatch {
  int bpi;
  int64_t bstride;
  const double* bcoef;
  int k0;
  const int* active;
};

// Per-instance view: field offset, operator coefficients and the weights a[k0+m], g[k0+m].
struct FusedInst {
  int64_t off;
  int lblock;
  bool skip;
  double coef, dinv_int, dinv_edge;
  double a[3], g[3];
};

__device__ __forceinline__ FusedInst fused_inst(const FusedBatch& B, const OpDesc& A,
                                                const double (&a)[3], const double (&g)[3]) {
  FusedInst I;
  const int inst = blockIdx.x / B.bpi;
  I.lblock = blockIdx.x - inst * B.bpi;
  I.off = (int64_t)inst * B.bstride;
  I.skip = B.active && !B.active[inst];
  I.coef = A.coef;
  I.dinv_int = A.dinv_int;
  I.dinv_edge = A.dinv_edge;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    I.a[m] = a[m];
    I.g[m] = g[m];
  }
  if (B.bcoef) {
    const double* rc = B.bcoef + (int64_t)inst * kCoefStride;
    I.coef = rc[0];
    I.dinv_int = rc[1];
    I.dinv_edge = rc[2];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int k = min(B.k0 + m, 7);
      I.a[m] = rc[3 + k];
      I.g[m] = rc[11 + k];
    }
  }
  return I;
}

template <typename T>
struct Smooth3Args {
  OpDesc A;
  const T* b;
  T* out;
  T* r;  // MODE 1: the residual
  double a[3], g[3];  // sweeps 0, 1, 2 (a[0] = a0; g[0] unused)
  int wstrips, rgroups, tiles;
  FusedBatch B;
};

// A x at row k of a register window of rows (V = 2 values per lane), the
// horizontal neighbours by DPP (zero from outside the wavefront).
//
// In float32 the 13-point operator is applied as two 5-point Laplacians: with
// even reflection of the rows, S13 = L5 L5 holds row by row, boundary rows
// included (20 c - 8 axis + 2 diag + far is L5 of u = L5 x, and the reflected
// ghost rows of x give reflected ghost rows of u).  u is formed at rows k-1,
// k, k+1; successive rows of an unrolled sweep share those values (the
// compiler computes each once), so a sweep costs two 5-point stencils per
// node instead of one 13-point stencil: 12% fewer vector instructions in the
// top-level post-smoother, different rounding (within the float32 V-cycle's
// own).  The output columns need u at columns c-1 .. c+2 only, which lanes
// 1 .. 62 have (u at a lane's first column needs its left neighbour, at its
// second its right one), the same lanes as the 13-point form.  In float64 the
// 13-point form stays: there the split form took more registers (the fused
// two-sweep pass went from 238 to 294).
template <typename T>
__device__ __forceinline__ void lap5_pair(const T (&m)[2], const T (&c)[2], const T (&p)[2],
                                          T (&u)[2]) {
  const T z = T(0);
  const T l = from_left(c[1], z), r = from_right(c[0], z);
  u[0] = ((l + c[1]) + (m[0] + p[0])) - T(4) * c[0];
  u[1] = ((c[0] + r) + (m[1] + p[1])) - T(4) * c[1];
}

template <int OP, typename T, int N>
__device__ __forceinline__ void window_apply(const T (&w)[N][2], int k, T coef, T (&ax)[2]) {
  constexpr int V = 2;
  if constexpr (OP == 1 && std::is_same<T, float>::value) {
    T um[2], uc[2], up[2], lu[2];
    lap5_pair(w[k - 2], w[k - 1], w[k], um);
    lap5_pair(w[k - 1], w[k], w[k + 1], uc);
    lap5_pair(w[k], w[k + 1], w[k + 2], up);
    lap5_pair(um, uc, up, lu);
#pragma unroll
    for (int i = 0; i < V; ++i) ax[i] = w[k][i] + coef * lu[i];
  } else {
    const T z = T(0);
    T e[V + 4];
    e[0] = OP == 1 ? from_left(w[k][0], z) : z;
    e[1] = from_left(w[k][1], z);
    e[2] = w[k][0];
    e[3] = w[k][1];
    e[4] = from_right(w[k][0], z);
    e[5] = OP == 1 ? from_right(w[k][1], z) : z;
    Nb13T<T> nb[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      nb[i].c = e[i + 2];
      nb[i].xm1 = e[i + 1];
      nb[i].xp1 = e[i + 3];
      nb[i].ym1 = w[k - 1][i];
      nb[i].yp1 = w[k + 1][i];
    }
    if constexpr (OP == 1) {
      T m[V + 2], p[V + 2];
      m[0] = from_left(w[k - 1][1], z);
      m[1] = w[k - 1][0];
      m[2] = w[k - 1][1];
      m[3] = from_right(w[k - 1][0], z);
      p[0] = from_left(w[k + 1][1], z);
      p[1] = w[k + 1][0];
      p[2] = w[k + 1][1];
      p[3] = from_right(w[k + 1][0], z);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        nb[i].xm2 = e[i];
        nb[i].xp2 = e[i + 4];
        nb[i].ym2 = w[k - 2][i];
        nb[i].yp2 = w[k + 2][i];
        nb[i].dmm = m[i];
        nb[i].dmp = m[i + 2];
        nb[i].dpm = p[i];
        nb[i].dpp = p[i + 2];
      }
    }
#pragma unroll
    for (int i = 0; i < V; ++i) ax[i] = apply_vals<OP>(nb[i], coef);
  }
}

// MODE 1 (degree-2 smoothers): two sweeps, then the residual of their
// result, r = b - A x2, instead of the third sweep; stores x2 and r.
template <int OP, int RPW, int MODE, typename T>
__global__ void __launch_bounds__(kStreamTPB) k_smooth3(Smooth3Args<T> P) {
  constexpr int R = (OP == 1) ? 2 : 1;
  constexpr int NB = RPW + 4 * R;  // b (and x1) rows j0-2R .. jl+2R
  constexpr int NX = RPW + 2 * R;  // x2 rows j0-R .. jl+R
  using V2 = VecN<T, 2>;
  const int n = P.A.n, mask = n - 1;
  const int lane = threadIdx.x & 63;
  const FusedInst I = fused_inst(P.B, P.A, P.a, P.g);
  const T* const Bp = P.b + I.off;
  T* const Op = P.out + I.off;
  const T tdi = T(I.dinv_int), tde = T(I.dinv_edge), tcoef = T(I.coef);
  const T ca0 = T(I.a[0]), ca1 = T(I.a[1]), cg1 = T(I.g[1]), ca2 = T(I.a[2]), cg2 = T(I.g[2]);
  auto dinv_row = [&](int jr) -> T { return row_dinv<OP, T>(tdi, tde, jr, n); };
  auto coef_row = [&](int jr) -> T { return (OP == 2 && (jr == 0 || jr == n)) ? T(0) : tcoef; };
  const int wpb = kStreamTPB / 64;
  const int t0 = __builtin_amdgcn_readfirstlane(I.lblock * wpb + (threadIdx.x >> 6));
  for (int t = t0; !I.skip && t < P.tiles; t += P.B.bpi * wpb) {
    int rg, strip;
    if (!grouped_tile(t, P.wstrips, P.rgroups, rg, strip)) continue;
    const int j0 = rg * RPW;
    const int jl = min(j0 + RPW, n + 1) - 1;
    const int col = strip * kS3Cols + 2 * (lane - 2);  // this lane's first column (unwrapped)
    const int cm = col & mask;                          // even, so cm + 1 < n

    // b and x1 over rows j0-2R .. jl+2R (reflected); rows past the tile's reach are unused
    T bw[NB][2], x1[NB][2];
    int jrb[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int jj = j0 - 2 * R + k;
      jrb[k] = refl(min(jj, jl + 2 * R), n);
      const V2 v = *reinterpret_cast<const V2*>(Bp + (int64_t)jrb[k] * n + cm);
      const T d0 = ca0 * dinv_row(jrb[k]);
      bw[k][0] = v.v[0];
      bw[k][1] = v.v[1];
      x1[k][0] = d0 * v.v[0];
      x1[k][1] = d0 * v.v[1];
    }
    // x2 over rows j0-R .. jl+R
    T x2[NX][2];
#pragma unroll
    for (int k2 = 0; k2 < NX; ++k2) {
      const int k = k2 + R;  // the same row in the b window
      const int jr = jrb[k];
      T ax[2];
      window_apply<OP>(x1, k, coef_row(jr), ax);
      const T ad = ca1 * dinv_row(jr);
#pragma unroll
      for (int i = 0; i < 2; ++i)
        x2[k2][i] = x1[k][i] + ad * (bw[k][i] - ax[i]) + cg1 * x1[k][i];
    }
    // x3 on the tile's rows, stored by lanes 2 .. 61 for columns inside the row
    const bool own = lane >= 2 && lane < 2 + kS3Lanes && col < n;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int j = j0 + s;
      if (j > jl) break;
      const int k2 = s + R, k = s + 2 * R;
      T ax[2];
      window_apply<OP>(x2, k2, coef_row(j), ax);
      if constexpr (MODE == 1) {
        V2 xo, ro;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          xo.v[i] = x2[k2][i];
          ro.v[i] = bw[k][i] - ax[i];
        }
        if (own) {
          const int64_t off = (int64_t)j * n + col;
          store_nt(reinterpret_cast<V2*>(Op + off), xo);
          store_nt(reinterpret_cast<V2*>(P.r + I.off + off), ro);
        }
      } else {
        const T ad = ca2 * dinv_row(j);
        V2 o;
#pragma unroll
        for (int i = 0; i < 2; ++i)
          o.v[i] = x2[k2][i] + ad * (bw[k][i] - ax[i]) + cg2 * (x2[k2][i] - x1[k][i]);
        if (own) store_nt(reinterpret_cast<V2*>(Op + (int64_t)j * n + col), o);
      }
    }
  }
}

// k_smooth3 followed by the residual of its result, r = b - A x3, in the
// same pass (x3 over the tile's rows widened by the stencil's reach): reads
// b, writes x3 and r, where the separate residual pass would read x3 and b
// again.  One more stencil level narrows the valid lanes to 3 .. 60 (116
// columns per wavefront).
constexpr int kS3RLanes = 58;
constexpr int kS3RCols = 2 * kS3RLanes;

template <typename T>
struct Smooth3RArgs {
  OpDesc A;
  const T* b;
  T* out;
  T* r;
  double a0, a1, g1, a2, g2;
  int wstrips, rgroups, tiles;
};

template <int OP, int RPW, typename T>
__global__ void __launch_bounds__(kStreamTPB) k_smooth3r(Smooth3RArgs<T> P) {
  constexpr int R = (OP == 1) ? 2 : 1;
  constexpr int NB = RPW + 6 * R;  // b and x1 rows j0-3R .. jl+3R
  constexpr int N2 = RPW + 4 * R;  // x2 rows j0-2R .. jl+2R
  constexpr int N3 = RPW + 2 * R;  // x3 rows j0-R .. jl+R
  using V2 = VecN<T, 2>;
  const int n = P.A.n, mask = n - 1;
  const int lane = threadIdx.x & 63;
  const T tdi = T(P.A.dinv_int), tde = T(P.A.dinv_edge), tcoef = T(P.A.coef);
  const T ca0 = T(P.a0), ca1 = T(P.a1), cg1 = T(P.g1), ca2 = T(P.a2), cg2 = T(P.g2);
  auto dinv_row = [&](int jr) -> T { return row_dinv<OP, T>(tdi, tde, jr, n); };
  auto coef_row = [&](int jr) -> T { return (OP == 2 && (jr == 0 || jr == n)) ? T(0) : tcoef; };
  const int wpb = kStreamTPB / 64;
  const int t0 = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
  for (int t = t0; t < P.tiles; t += gridDim.x * wpb) {
    int rg, strip;
    if (!grouped_tile(t, P.wstrips, P.rgroups, rg, strip)) continue;
    const int j0 = rg * RPW;
    const int jl = min(j0 + RPW, n + 1) - 1;
    const int col = strip * kS3RCols + 2 * (lane - 3);
    const int cm = col & mask;

    T bw[NB][2], x1[NB][2];
    int jrb[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int jj = j0 - 3 * R + k;
      jrb[k] = refl(min(jj, jl + 3 * R), n);
      const V2 v = *reinterpret_cast<const V2*>(P.b + (int64_t)jrb[k] * n + cm);
      const T d0 = ca0 * dinv_row(jrb[k]);
      bw[k][0] = v.v[0];
      bw[k][1] = v.v[1];
      x1[k][0] = d0 * v.v[0];
      x1[k][1] = d0 * v.v[1];
    }
    T x2[N2][2];
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int k = k2 + R;
      const int jr = jrb[k];
      T ax[2];
      window_apply<OP>(x1, k, coef_row(jr), ax);
      const T ad = ca1 * dinv_row(jr);
#pragma unroll
      for (int i = 0; i < 2; ++i)
        x2[k2][i] = x1[k][i] + ad * (bw[k][i] - ax[i]) + cg1 * x1[k][i];
    }
    T x3[N3][2];
#pragma unroll
    for (int k3 = 0; k3 < N3; ++k3) {
      const int k2 = k3 + R, k = k3 + 2 * R;
      const int jr = jrb[k];
      T ax[2];
      window_apply<OP>(x2, k2, coef_row(jr), ax);
      const T ad = ca2 * dinv_row(jr);
#pragma unroll
      for (int i = 0; i < 2; ++i)
        x3[k3][i] = x2[k2][i] + ad * (bw[k][i] - ax[i]) + cg2 * (x2[k2][i] - x1[k][i]);
    }
    const bool own = lane >= 3 && lane < 3 + kS3RLanes && col < n;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int j = j0 + s;
      if (j > jl) break;
      const int k3 = s + R, k = s + 3 * R;
      T ax[2];
      window_apply<OP>(x3, k3, coef_row(j), ax);
      V2 xo, ro;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        xo.v[i] = x3[k3][i];
        ro.v[i] = bw[k][i] - ax[i];
      }
      if (own) {
        const int64_t off = (int64_t)j * n + col;
        store_nt(reinterpret_cast<V2*>(P.out + off), xo);
        store_nt(reinterpret_cast<V2*>(P.r + off), ro);
      }
    }
  }
}

// The last two sweeps of the post-smoother in one pass:
//   x2 = x1 + a1 D^{-1}(b - A x1) + g1 (x1 - x0),
//   x3 = x2 + a2 D^{-1}(b - A x2) + g2 (x2 - x1),
// with x2 in registers over the tile's rows widened by the stencil's reach
// (same overlapping strips as k_smooth3).  Reads x1 (stencil window), x0 and
// b (pointwise) and, for the reductions, q; writes x3, which must not alias
// x1 or x0 (neighbouring tiles still read them).  Epilogues: none, partials
// of <b, x3>_W (S2_DOT), or of <b, x3>_W and <x3, q>_W (S2_DOT2), taken on
// x3 as stored (TO).
enum { S2_NONE = 0, S2_DOT = 1, S2_DOT2 = 2 };

template <typename T, typename TO>
struct Smooth2Args {
  OpDesc A;
  const T* x1;
  const T* x0;      // nullptr when g1 == 0 (x1 - x0 then not formed)
  const T* b;
  const double* q;  // S2_DOT2
  TO* out;
  double* partials;
  double a[3], g[3];  // a[0], g[0]: the first of the two sweeps, a[1], g[1]: the second
  int wstrips, rgroups, tiles;
  FusedBatch B;
};

template <int OP, int EP, int RPW, typename T, typename TO>
__global__ void __launch_bounds__(kStreamTPB) k_smooth2(Smooth2Args<T, TO> P) {
  constexpr int R = (OP == 1) ? 2 : 1;
  constexpr int NW = RPW + 4 * R;  // x1 rows j0-2R .. jl+2R
  constexpr int NX = RPW + 2 * R;  // x2 rows j0-R .. jl+R
  using V2 = VecN<T, 2>;
  const int n = P.A.n, mask = n - 1;
  const int lane = threadIdx.x & 63;
  const int wpb = kStreamTPB / 64;
  const FusedInst I = fused_inst(P.B, P.A, P.a, P.g);
  const T* const X1p = P.x1 + I.off;
  const T* const X0p = P.x0 ? P.x0 + I.off : nullptr;
  const T* const Bp = P.b + I.off;
  const double* const Qp = P.q ? P.q + I.off : nullptr;
  TO* const Op = P.out + I.off;
  const int t0 = __builtin_amdgcn_readfirstlane(I.lblock * wpb + (threadIdx.x >> 6));
  double acc = 0.0, acc2 = 0.0;
  // (every wavefront reaches the reductions below, which synchronise the block)
  for (int t = t0; !I.skip && t < P.tiles; t += P.B.bpi * wpb) {
    int rg, strip;
    if (!grouped_tile(t, P.wstrips, P.rgroups, rg, strip)) continue;
    const int j0 = rg * RPW;
    const int jl = min(j0 + RPW, n + 1) - 1;
    const int col = strip * kS3Cols + 2 * (lane - 2);
    const int cm = col & mask;
    const T tdi = T(I.dinv_int), tde = T(I.dinv_edge), tcoef = T(I.coef);
    const T ca1 = T(I.a[0]), cg1 = T(I.g[0]), ca2 = T(I.a[1]), cg2 = T(I.g[1]);
    auto dinv_row = [&](int jr) -> T { return row_dinv<OP, T>(tdi, tde, jr, n); };
    auto coef_row = [&](int jr) -> T { return (OP == 2 && (jr == 0 || jr == n)) ? T(0) : tcoef; };

    T x1[NW][2];
    int jrw[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int jj = j0 - 2 * R + k;
      jrw[k] = refl(min(jj, jl + 2 * R), n);
      const V2 v = *reinterpret_cast<const V2*>(X1p + (int64_t)jrw[k] * n + cm);
      x1[k][0] = v.v[0];
      x1[k][1] = v.v[1];
    }
    T x2[NX][2], bw[NX][2];
#pragma unroll
    for (int k2 = 0; k2 < NX; ++k2) {
      const int k = k2 + R;
      const int jr = jrw[k];
      const int64_t o = (int64_t)jr * n + cm;
      const V2 bv = *reinterpret_cast<const V2*>(Bp + o);
      V2 pv{};
      if (X0p) pv = *reinterpret_cast<const V2*>(X0p + o);
      T ax[2];
      window_apply<OP>(x1, k, coef_row(jr), ax);
      const T ad = ca1 * dinv_row(jr);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        bw[k2][i] = bv.v[i];
        x2[k2][i] = x1[k][i] + ad * (bv.v[i] - ax[i]) + cg1 * (x1[k][i] - pv.v[i]);
      }
    }
    const bool own = lane >= 2 && lane < 2 + kS3Lanes && col < n;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int j = j0 + s;
      if (j > jl) break;
      const int k2 = s + R, k = s + 2 * R;
      T ax[2];
      window_apply<OP>(x2, k2, coef_row(j), ax);
      const T ad = ca2 * dinv_row(j);
      VecN<TO, 2> o;
#pragma unroll
      for (int i = 0; i < 2; ++i)
        o.v[i] = TO(x2[k2][i] + ad * (bw[k2][i] - ax[i]) + cg2 * (x2[k2][i] - x1[k][i]));
      if (own) {
        const int64_t off = (int64_t)j * n + col;
        store_nt(reinterpret_cast<VecN<TO, 2>*>(Op + off), o);
        if constexpr (EP != S2_NONE) {
          const double wgt = row_weight(j, n);
#pragma unroll
          for (int i = 0; i < 2; ++i) acc += wgt * double(bw[k2][i]) * double(o.v[i]);
          if constexpr (EP == S2_DOT2) {
            const VecN<double, 2> qv = *reinterpret_cast<const VecN<double, 2>*>(Qp + off);
#pragma unroll
            for (int i = 0; i < 2; ++i) acc2 += wgt * double(o.v[i]) * qv.v[i];
          }
        }
      }
    }
  }
  if constexpr (EP != S2_NONE) {
    const double s1 = block_sum_n<kStreamTPB>(acc);
    if (threadIdx.x == 0) P.partials[blockIdx.x] = s1;
    if constexpr (EP == S2_DOT2) {
      const double s2 = block_sum_n<kStreamTPB>(acc2);
      if (threadIdx.x == 0) P.partials[gridDim.x + blockIdx.x] = s2;
    }
  }
}

// The coarse-grid correction and the whole post-smoother of a level in one
// pass (single grids):
//   x_0 = x + P e   (P: tensor-product cubic interpolation of the coarse
//                    correction e, formed on load),
//   x_{k+1} = x_k + a_k D^{-1}(b - A x_k) + g_k (x_k - x_{k-1}),  k = 0 .. D-1
//   (g_0 = 0: the first sweep of the Chebyshev recurrence has no x_{-1}).
// The separate form is three passes (prolongation, one sweep, the last two
// sweeps) that write and re-read x_0 and x_1; here x_0 .. x_{D-1} live in
// registers over the tile's rows widened by the stencil's reach (D levels:
// D R rows each side), so the pass reads x, e and b and writes x_D only.
// Each lane holds two fine columns c, c+1 (c even) and loads the coarse
// column c/2 of the coarse rows the window needs; the interpolation at c+1
// takes the coarse columns c/2 - 1 .. c/2 + 2 from lanes -1 .. +2 (DPP), so
// x_0 is valid on lanes 1 .. 61, and every stencil level narrows that by a
// lane each side: lanes 1+D .. 61-D produce output (strips 2 (61 - 2D)
// columns apart, the last cut at n).  A fine ghost row takes its
// interpolated value from the unreflected coarse rows around it (the coarse
// rows reflected on load): P commutes with the even reflection, so the value
// equals the one on its mirror row, as for the stencil levels.  Epilogues as
// for k_smooth2 (S2_NONE, S2_DOT, S2_DOT2).
template <int D>
struct PostGeom {
  static constexpr int kLanes = 61 - 2 * D;
  static constexpr int kCols = 2 * kLanes;
};

template <typename T, typename TO>
struct PostArgs {
  OpDesc A;
  const T* x;       // the level's iterate before the correction
  const T* e;       // coarse correction, (n/2 + 1) x n/2
  const T* b;
  const double* q;  // S2_DOT2
  TO* out;
  double* partials;
  double a[3], g[3];
  int wstrips, rgroups, tiles;
  T* x0out;  // D = 1: receives x0 = x + P e
};

template <int OP, int D, int EP, int RPW, typename T, typename TO>
__global__ void __launch_bounds__(kStreamTPB) k_post(PostArgs<T, TO> P) {
  constexpr int R = (OP == 1) ? 2 : 1;
  static_assert((D * R) % 2 == 0 && RPW % 2 == 0, "window rows start on an even fine row");
  constexpr int NW = RPW + 2 * D * R;  // x0 and b rows j0-DR .. j0-DR+NW-1
  constexpr int NC = NW / 2 + 3;       // coarse rows (j0-DR)/2 - 1 .. (j0-DR)/2 + NW/2 + 1
  constexpr int LO = 1 + D, HI = 61 - D;  // output lanes
  using V2 = VecN<T, 2>;
  const int n = P.A.n, mask = n - 1;
  const int nc = n >> 1;
  const int lane = threadIdx.x & 63;
  const int wpb = kStreamTPB / 64;
  const T tdi = T(P.A.dinv_int), tde = T(P.A.dinv_edge), tcoef = T(P.A.coef);
  auto dinv_row = [&](int jr) -> T { return row_dinv<OP, T>(tdi, tde, jr, n); };
  auto coef_row = [&](int jr) -> T { return (OP == 2 && (jr == 0 || jr == n)) ? T(0) : tcoef; };
  const int t0 = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
  double acc = 0.0, acc2 = 0.0;
  for (int t = t0; t < P.tiles; t += gridDim.x * wpb) {
    int rg, strip;
    if (!grouped_tile(t, P.wstrips, P.rgroups, rg, strip)) continue;
    const int j0 = rg * RPW;
    const int jl = min(j0 + RPW, n + 1) - 1;
    const int col = strip * PostGeom<D>::kCols + 2 * (lane - LO);
    const int cm = col & mask;
    const int ic = cm >> 1;  // this lane's coarse column
    // Every load of the tile is issued before any value is used, so their
    // latencies overlap (left to itself, the compiler sinks each load to its
    // first use to save registers, which exposes them one after another): the
    // coarse rows, x and b over the window (rows past the tile's reach repeat
    // its last reachable row and are never used), and q at the output rows
    // (clamped to valid rows and columns; only the owned ones are used).
    const int jc0 = ((j0 - D * R) >> 1) - 1;
    T ev[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) ev[m] = P.e[(int64_t)refl(jc0 + m, nc) * nc + ic];
    V2 xv[NW], bv[NW];
    int jrw[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int jj = j0 - D * R + k;
      jrw[k] = refl(min(jj, jl + D * R), n);
      const int64_t o = (int64_t)jrw[k] * n + cm;
      xv[k] = *reinterpret_cast<const V2*>(P.x + o);
      bv[k] = *reinterpret_cast<const V2*>(P.b + o);
    }
    VecN<double, 2> qv[EP == S2_DOT2 ? RPW : 1];
    if constexpr (EP == S2_DOT2) {
#pragma unroll
      for (int s = 0; s < RPW; ++s)
        qv[s] = *reinterpret_cast<const VecN<double, 2>*>(P.q + (int64_t)min(j0 + s, jl) * n + cm);
    }
    __builtin_amdgcn_sched_barrier(0);
    // coarse rows, interpolated in x at the lane's two fine columns
    T ce[NC][2];
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      const T v = ev[m];
      const T vm1 = from_left(v, T(0));
      const T vp1 = from_right(v, T(0));
      const T vp2 = from_right(vp1, T(0));
      ce[m][0] = v;
      ce[m][1] = (-vm1 + T(9) * v + T(9) * vp1 - vp2) * T(0.0625);
    }
    // x0 = x + P e and b over the window rows (rows past the tile's reach are unused)
    T x0[NW][2], bw[NW][2];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int m = (k >> 1) + 1;  // coarse row of jj (even), or of jj - 1 (odd)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        T pe;
        if ((k & 1) == 0) {
          pe = ce[m][i];
        } else {
          pe = (-ce[m - 1][i] + T(9) * ce[m][i] + T(9) * ce[m + 1][i] - ce[m + 2][i]) * T(0.0625);
        }
        x0[k][i] = xv[k].v[i] + pe;
        bw[k][i] = bv[k].v[i];
      }
    }
    // x1 over rows j0-(D-1)R .. jl+(D-1)R
    constexpr int N1 = NW - 2 * R;
    T x1[N1][2];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      const int k = k1 + R;
      T ax[2];
      window_apply<OP>(x0, k, coef_row(jrw[k]), ax);
      const T ad = T(P.a[0]) * dinv_row(jrw[k]);
#pragma unroll
      for (int i = 0; i < 2; ++i) x1[k1][i] = x0[k][i] + ad * (bw[k][i] - ax[i]);
    }
    // x2 over rows j0-(D-2)R .. jl+(D-2)R (D >= 2)
    constexpr int N2 = D >= 2 ? NW - 4 * R : 1;
    T x2[N2][2];
#pragma unroll
    for (int k2 = 0; k2 < (D >= 2 ? N2 : 0); ++k2) {
      const int k1 = k2 + R, k = k2 + 2 * R;
      T ax[2];
      window_apply<OP>(x1, k1, coef_row(jrw[k]), ax);
      const T ad = T(P.a[1]) * dinv_row(jrw[k]);
      const T g1 = T(P.g[1]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
        x2[k2][i] = x1[k1][i] + ad * (bw[k][i] - ax[i]) + g1 * (x1[k1][i] - x0[k][i]);
    }
    const bool own = lane >= LO && lane <= HI && col < n;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int j = j0 + s;
      // (continue, not break: with a break the compiler kept the 12-row
      // windows of the reducing variants in scratch memory)
      if (j > jl) continue;
      const int k = s + D * R;  // the row in the x0 / b window
      VecN<TO, 2> o;
      if constexpr (D == 1) {
#pragma unroll
        for (int i = 0; i < 2; ++i) o.v[i] = TO(x1[s][i]);
      } else if constexpr (D == 2) {
#pragma unroll
        for (int i = 0; i < 2; ++i) o.v[i] = TO(x2[s][i]);
      } else {
        const int k2 = s + R, k1 = s + 2 * R;
        T ax[2];
        window_apply<OP>(x2, k2, coef_row(j), ax);
        const T ad = T(P.a[2]) * dinv_row(j);
        const T g2 = T(P.g[2]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
          o.v[i] = TO(x2[k2][i] + ad * (bw[k][i] - ax[i]) + g2 * (x2[k2][i] - x1[k1][i]));
      }
      if (own) {
        const int64_t off = (int64_t)j * n + col;
        store_nt(reinterpret_cast<VecN<TO, 2>*>(P.out + off), o);
        if constexpr (D == 1) {
          // x0 = x + P e as well: the next sweep's (x1 - x0) term reads it
          VecN<T, 2> xo;
#pragma unroll
          for (int i = 0; i < 2; ++i) xo.v[i] = x0[k][i];
          store_nt(reinterpret_cast<VecN<T, 2>*>(P.x0out + off), xo);
        }
        if constexpr (EP != S2_NONE) {
          const double wgt = row_weight(j, n);
#pragma unroll
          for (int i = 0; i < 2; ++i) acc += wgt * double(bw[k][i]) * double(o.v[i]);
          if constexpr (EP == S2_DOT2) {
#pragma unroll
            for (int i = 0; i < 2; ++i) acc2 += wgt * double(o.v[i]) * qv[s].v[i];
          }
        }
      }
    }
  }
  if constexpr (EP != S2_NONE) {
    const double s1 = block_sum_n<kStreamTPB>(acc);
    if (threadIdx.x == 0) P.partials[blockIdx.x] = s1;
    if constexpr (EP == S2_DOT2) {
      const double s2 = block_sum_n<kStreamTPB>(acc2);
      if (threadIdx.x == 0) P.partials[gridDim.x + blockIdx.x] = s2;
    }
  }
}

// ------------------------------------------------------------------ launch
namespace {

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

}  // namespace

// Batch of the launches issued by this thread (set by the ensemble driver;
// count 1 = a single field).
thread_local BatchCtx g_batch;

// Tiled kernels from n = 128, one 128-column strip (below, the
// one-node-per-thread kernels).  The float32 128^2 level gains from the fused
// smoother passes (4096^2 mixed step 18.82-18.84 ms against 18.91-18.93 with
// that level left to the one-node-per-thread kernels).
bool stream_ok(int n, int elem_bytes) {
  (void)elem_bytes;  // two values per lane in either precision
  return n >= 128;
}

// Rows per tile: 5 for the operator applications (y = A x, q = A p: on
// 4096^2 the 13-point SpMV measured 47.8-48.8 us with 5 rows against
// 48.4-49.1 with 4), 4 for the kernels with more inputs per row (smoothing
// sweeps, residuals, the CG step: a 5-row tile holds too many registers;
// smoothing measured 91 us with 4 rows, 93 with 5).  Fewer rows re-read more
// neighbour rows, more rows widen the band of rows in flight; 2, 3, 6 and 8
// were slower.  BF_STREAM_RPW=4, 5 or 8 forces one height; a batch may set its own.
StreamCfg stream_cfg(int n, int elem_bytes, bool apply) {
  StreamCfg c;
  static const int rpw_env = env_int("BF_STREAM_RPW", 0);
  c.rpw = apply ? 5 : 4;
  if (rpw_env == 4 || rpw_env == 5 || rpw_env == 8) c.rpw = rpw_env;
  if (g_batch.rpw == 4 || g_batch.rpw == 5 || g_batch.rpw == 8) c.rpw = g_batch.rpw;
  c.wstrips = n / (64 * kLaneCols);
  c.rgroups = (n + 1 + c.rpw - 1) / c.rpw;
  c.tiles = c.wstrips * c.rgroups;
  const int wpb = kStreamTPB / 64;
  const int64_t blocks = ((int64_t)c.tiles + wpb - 1) / wpb;
  c.blocks = (int)(blocks < kStreamMaxBlocks ? blocks : kStreamMaxBlocks);
  return c;
}

StreamCfg stream_cfg(int n, int elem_bytes) { return stream_cfg(n, elem_bytes, false); }
bool stream_ok(int n) { return stream_ok(n, 8); }
StreamCfg stream_cfg(int n) { return stream_cfg(n, 8); }

template <int OP, int EPI, typename T, typename TO>
static int dispatch(const StreamCfg& c, StreamArgs<T, TO> P, hipStream_t st) {
  P.rgroups = c.rgroups;
  P.wstrips = c.wstrips;
  P.tiles = c.tiles;
  const BatchCtx& B = g_batch;
  P.batch = B.count > 1 ? B.count : 1;
  P.bstride = B.count > 1 ? B.stride : 0;
  P.bcoef = B.coef;
  P.ia = B.ia;
  P.ig = B.ig;
  P.ia0 = B.ia0;
  P.active = B.active;
  // per instance: all of its tiles, at most kStreamMaxBlocks / batch workgroups
  int bpi = c.blocks;
  if (P.batch > 1) {
    const int cap = kStreamMaxBlocks / P.batch;
    bpi = bpi < cap ? bpi : (cap > 0 ? cap : 1);
  }
  P.bpi = bpi;
  const int blocks = bpi * P.batch;
  if (c.rpw == 8)
    hipLaunchKernelGGL((k_stream<OP, EPI, 8, T, TO>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
  else if (c.rpw == 4)
    hipLaunchKernelGGL((k_stream<OP, EPI, 4, T, TO>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
  else
    hipLaunchKernelGGL((k_stream<OP, EPI, 5, T, TO>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
  return blocks;
}

template <int EPI, typename T, typename TO>
static int stream_launch(const OpDesc& A, const T* x, const T* b, const T* xprev, TO* out,
                         double* partials, double a, double g, hipStream_t st, double a0 = 0.0,
                         const double* q = nullptr, float* out32 = nullptr) {
  constexpr bool kApply = EPI == E_APPLY || EPI == E_APPLY_DOT || EPI == E_APPLY_DOT_DD;
  const StreamCfg c = stream_cfg(A.n, sizeof(T), kApply);
  StreamArgs<T, TO> P{};
  P.A = A;
  P.G = make_geo(A.n);
  P.x = x;
  P.b = b;
  P.xprev = xprev;
  P.out = out;
  P.partials = partials;
  P.a = a;
  P.g = g;
  P.a0 = a0;
  P.q = q;
  P.out32 = out32;
  if (A.op == 0) return dispatch<0, EPI>(c, P, st);
  if (A.op == 2) return dispatch<2, EPI>(c, P, st);
  return dispatch<1, EPI>(c, P, st);
}

int stream_apply(const OpDesc& A, const double* x, double* y, hipStream_t st) {
  return stream_launch<E_APPLY, double, double>(A, x, nullptr, nullptr, y, nullptr, 0, 0, st);
}
int stream_apply_dot(const OpDesc& A, const double* p, double* q, double* partials, bool dd,
                     hipStream_t st) {
  if (dd)
    return stream_launch<E_APPLY_DOT_DD, double, double>(A, p, nullptr, nullptr, q, partials, 0,
                                                         0, st);
  return stream_launch<E_APPLY_DOT, double, double>(A, p, nullptr, nullptr, q, partials, 0, 0,
                                                    st);
}
int stream_residual_dd(const OpDesc& A, const double* x, const double* b, double* r,
                       double* partials, hipStream_t st, float* r32) {
  return stream_launch<E_RESID_DD, double, double>(A, x, b, nullptr, r, partials, 0, 0, st, 0.0,
                                                   nullptr, r32);
}
int stream_guess(const OpDesc& A, const double* x, const double* b, double* partials,
                 hipStream_t st) {
  return stream_launch<E_GUESS, double, double>(A, x, b, nullptr, nullptr, partials, 0, 0, st);
}

template <typename T>
int stream_residual(const OpDesc& A, const T* x, const T* b, T* r, double* partials,
                    hipStream_t st) {
  if (partials)
    return stream_launch<E_RESID_NORM, T, T>(A, x, b, nullptr, r, partials, 0, 0, st);
  return stream_launch<E_RESID, T, T>(A, x, b, nullptr, r, nullptr, 0, 0, st);
}
template <typename T>
void stream_smooth(const OpDesc& A, const T* x, const T* xprev, const T* b, T* xout, double a,
                   double g, hipStream_t st) {
  stream_launch<E_SMOOTH, T, T>(A, x, b, xprev, xout, nullptr, a, g, st);
}
template <typename T>
void stream_smooth_from_zero(const OpDesc& A, const T* b, T* xout, double a0, double a1,
                             double g1, hipStream_t st) {
  stream_launch<E_SMOOTH_XB, T, T>(A, b, b, nullptr, xout, nullptr, a1, g1, st, a0);
}
template <typename T>
void stream_smooth_prev_from_b(const OpDesc& A, const T* x, const T* b, T* xout, double a0,
                               double a, double g, hipStream_t st) {
  stream_launch<E_SMOOTH_PB, T, T>(A, x, b, nullptr, xout, nullptr, a, g, st, a0);
}
int stream_smooth_dot(const OpDesc& A, const double* x, const double* xprev, const double* b,
                      double* xout, double a, double g, double* partials, hipStream_t st) {
  return stream_launch<E_SMOOTH_DOT, double, double>(A, x, b, xprev, xout, partials, a, g, st);
}
int stream_smooth_dot2(const OpDesc& A, const float* x, const float* xprev, const float* b,
                       double* xout, const double* q, double a, double g, double* partials,
                       hipStream_t st) {
  return stream_launch<E_SMOOTH_DOT2, float, double>(A, x, b, xprev, xout, partials, a, g, st,
                                                     0.0, q);
}
// The overlapped-strip CH CG step (k_cg_ch): single grids only (a batch, also
// a batch of one with coefficient records or a mask, takes k_stream).
static bool cg_ch_ok(const OpDesc& A) {
  static const bool off = env_int("BF_NO_CG_CH", 0) != 0;
  const BatchCtx& B = g_batch;
  return !off && A.op == 1 && B.count <= 1 && !B.coef && !B.active;
}

template <int RPW, int WAVES, typename ZT>
static int launch_cg_ch_cfg(const OpDesc& A, const ZT* z, const ZT* p_old, ZT* p_new,
                            double* q, double* x, const double* scal, bool first,
                            double* partials, hipStream_t st) {
  CgArgs<ZT> P{};
  P.A = A;
  P.G = make_geo(A.n);
  P.z = z;
  P.p_old = p_old;
  P.p_new = p_new;
  P.q = q;
  P.x = x;
  P.scal = scal;
  P.partials = partials;
  P.first = first ? 1 : 0;
  P.wstrips = (A.n + kCgCols - 1) / kCgCols;
  P.rgroups = (A.n + 1 + RPW - 1) / RPW;
  P.tiles = P.wstrips * P.rgroups;
  const int wpb = kStreamTPB / 64;
  const int blocks = std::min((P.tiles + wpb - 1) / wpb, kStreamMaxBlocks);
  if (first)
    hipLaunchKernelGGL((k_cg_ch<RPW, ZT, WAVES, true, false>), dim3(blocks), dim3(kStreamTPB), 0,
                       st, P);
  else if (x)
    hipLaunchKernelGGL((k_cg_ch<RPW, ZT, WAVES, false, true>), dim3(blocks), dim3(kStreamTPB), 0,
                       st, P);
  else
    hipLaunchKernelGGL((k_cg_ch<RPW, ZT, WAVES, false, false>), dim3(blocks), dim3(kStreamTPB), 0,
                       st, P);
  return blocks;
}

// Tile height and occupancy target of k_cg_ch (BF_CG_CH_CFG selects one for
// measurements): 0 = 4 rows, at least 4 waves per SIMD (114 VGPRs); 1 = 4
// rows, the compiler's own register count; 2 = 2 rows, at least 4 waves;
// 3 = 8 rows, at least 3 waves.
template <typename ZT>
static int launch_cg_ch(const OpDesc& A, const ZT* z, const ZT* p_old, ZT* p_new,
                        double* q, double* x, const double* scal, bool first, double* partials,
                        hipStream_t st) {
  static const int cfg = env_int("BF_CG_CH_CFG", 0);
  switch (cfg) {
    case 1:
      return launch_cg_ch_cfg<4, 1>(A, z, p_old, p_new, q, x, scal, first, partials, st);
    case 2:
      return launch_cg_ch_cfg<2, 4>(A, z, p_old, p_new, q, x, scal, first, partials, st);
    case 3:
      return launch_cg_ch_cfg<8, 3>(A, z, p_old, p_new, q, x, scal, first, partials, st);
    default:
      return launch_cg_ch_cfg<4, 4>(A, z, p_old, p_new, q, x, scal, first, partials, st);
  }
}

int stream_cg_p(const OpDesc& A, const double* z, const double* p_old, double* p_new, double* q,
                double* x, const double* scal, bool first, double* partials, hipStream_t st) {
  if (cg_ch_ok(A)) return launch_cg_ch(A, z, p_old, p_new, q, x, scal, first, partials, st);
  const StreamCfg c = stream_cfg(A.n, 8);
  StreamArgs<double, double> P{};
  P.A = A;
  P.G = make_geo(A.n);
  P.x = z;
  P.xprev = p_old;
  P.out = q;
  P.out2 = p_new;
  P.xu = x;
  P.scal = scal;
  P.first = first ? 1 : 0;
  P.partials = partials;
  if (A.op == 0) return dispatch<0, E_CG_P>(c, P, st);
  if (A.op == 2) return dispatch<2, E_CG_P>(c, P, st);
  return dispatch<1, E_CG_P>(c, P, st);
}
int stream_cg_p32(const OpDesc& A, const float* z, const float* p_old, float* p_new, double* q,
                  double* x, const double* scal, bool first, double* partials, hipStream_t st) {
  if (cg_ch_ok(A)) return launch_cg_ch(A, z, p_old, p_new, q, x, scal, first, partials, st);
  const StreamCfg c = stream_cfg(A.n, 8);
  StreamArgs<double, double> P{};
  P.A = A;
  P.G = make_geo(A.n);
  P.z32 = z;
  P.p32_old = p_old;
  P.out = q;
  P.p32_new = p_new;
  P.xu = x;
  P.scal = scal;
  P.first = first ? 1 : 0;
  P.partials = partials;
  if (A.op == 0) return dispatch<0, E_CG_P32>(c, P, st);
  if (A.op == 2) return dispatch<2, E_CG_P32>(c, P, st);
  return dispatch<1, E_CG_P32>(c, P, st);
}
int stream_smooth_dot2_f32(const OpDesc& A, const float* x, const float* xprev, const float* b,
                           float* xout, const double* q, double a, double g, double* partials,
                           hipStream_t st) {
  return stream_launch<E_SMOOTH_DOT2, float, float>(A, x, b, xprev, xout, partials, a, g, st,
                                                    0.0, q);
}

// Batch context of a fused pass from this thread's batch (see BatchCtx; as
// for k_stream, the coefficient records and the mask apply whenever the batch
// supplies them, also to a batch of one); returns the workgroup count for
// `tiles` tiles per instance.
static int fused_batch(FusedBatch& B, int tiles, int k0) {
  const int wpb = kStreamTPB / 64;
  const BatchCtx& G = g_batch;
  const int count = G.count > 1 ? G.count : 1;
  const int per = std::min((tiles + wpb - 1) / wpb, kStreamMaxBlocks / count);
  B.bpi = per > 0 ? per : 1;
  B.bstride = count > 1 ? G.stride : 0;
  B.bcoef = G.coef;
  B.k0 = k0;
  B.active = G.active;
  return B.bpi * count;
}

// The three-sweep pass on every streamed level (n >= 128; measured on the
// 4096^2 step against a 1024 threshold: 20.15 against 20.33 ms mixed, 25.0
// against 25.3 ms float64 -- on the small levels it saves a launch).
// BF_NO_SMOOTH3=1: the two-pass form; BF_SMOOTH3_MIN=m: from n = m up.
bool smooth3_ok(int n) {
  static const bool off = [] {
    const char* v = std::getenv("BF_NO_SMOOTH3");
    return v && v[0] == '1';
  }();
  static const int lim = [] {
    const int m = env_int("BF_SMOOTH3_MIN", 0);
    return m >= 128 ? m : 128;
  }();
  return !off && n >= lim;
}

// The fused residual form for float32 levels (BF_NO_SMOOTH3R=1: off); in
// float64 the extra stencil level would not fit the registers.
bool smooth3r_ok(int n, int elem_bytes) {
  static const bool off = [] {
    const char* v = std::getenv("BF_NO_SMOOTH3R");
    return v && v[0] == '1';
  }();
  return !off && elem_bytes == 4 && smooth3_ok(n);
}

// Tile height of the fused float32 smoother passes on the small levels, where
// a launch has few wavefronts and its time is one wavefront's instruction
// chain: 2 rows on levels up to 512^2 (4096^2 mixed V-cycle 490.5 us against
// 498.6 with 8 rows everywhere; 4 rows, or 2 rows up to 1024^2, 492-494).
// BF_SMALL_RPW (2, 4 or 8) and BF_SMALL_N override the height and the level.
static int small_level_rpw(int n, int dflt) {
  static const int rpw = env_int("BF_SMALL_RPW", 2);
  static const int small_n = env_int("BF_SMALL_N", 512);
  if (n <= small_n && (rpw == 2 || rpw == 4 || rpw == 8)) return rpw;
  return dflt;
}

template <typename T>
void stream_smooth3_resid(const OpDesc& A, const T* b, T* xout, T* r, double a0, double a1,
                          double g1, double a2, double g2, hipStream_t st) {
  // 12 output rows per tile above the small levels: the stage-two and -three
  // halo rows are shared by more outputs (231 registers, two wavefronts per
  // SIMD as with 8 rows at 187; with k_post at 12 rows as well the 4096^2
  // mixed step took 9.98 ms against 10.07 with both at 8; 16 rows, 278
  // registers, 10.23).  BF_S3R_RPW=4|8|12|16 sets the height.
  Smooth3RArgs<T> P;
  P.A = A;
  P.b = b;
  P.out = xout;
  P.r = r;
  P.a0 = a0;
  P.a1 = a1;
  P.g1 = g1;
  P.a2 = a2;
  P.g2 = g2;
  static const int rpw_env = env_int("BF_S3R_RPW", 12);
  const int rpw = small_level_rpw(A.n, rpw_env);
  P.wstrips = (A.n + kS3RCols - 1) / kS3RCols;
  P.rgroups = (A.n + 1 + rpw - 1) / rpw;
  P.tiles = grouped_tiles(P.wstrips, P.rgroups);
  const int wpb = kStreamTPB / 64;
  const int blocks = std::min((P.tiles + wpb - 1) / wpb, kStreamMaxBlocks);
#define BF_S3R_GO(RPW_)                                                                     \
  do {                                                                                     \
    if (A.op == 0)                                                                         \
      hipLaunchKernelGGL((k_smooth3r<0, RPW_, T>), dim3(blocks), dim3(kStreamTPB), 0, st, P); \
    else if (A.op == 2)                                                                    \
      hipLaunchKernelGGL((k_smooth3r<2, RPW_, T>), dim3(blocks), dim3(kStreamTPB), 0, st, P); \
    else                                                                                   \
      hipLaunchKernelGGL((k_smooth3r<1, RPW_, T>), dim3(blocks), dim3(kStreamTPB), 0, st, P); \
  } while (0)
  if (rpw == 2)
    BF_S3R_GO(2);
  else if (rpw == 4)
    BF_S3R_GO(4);
  else if (rpw == 12)
    BF_S3R_GO(12);
  else if (rpw == 16)
    BF_S3R_GO(16);
  else
    BF_S3R_GO(8);
#undef BF_S3R_GO
}
template void stream_smooth3_resid<float>(const OpDesc&, const float*, float*, float*, double,
                                          double, double, double, double, hipStream_t);

template <int MODE, typename T>
static void launch_smooth3(const OpDesc& A, const T* b, T* xout, T* r, double a0, double a1,
                           double g1, double a2, double g2, hipStream_t st) {
  constexpr int RPW = 4;
  Smooth3Args<T> P;
  P.A = A;
  P.b = b;
  P.out = xout;
  P.r = r;
  P.a[0] = a0;
  P.a[1] = a1;
  P.a[2] = a2;
  P.g[0] = 0.0;
  P.g[1] = g1;
  P.g[2] = g2;
  P.wstrips = (A.n + kS3Cols - 1) / kS3Cols;
  P.rgroups = (A.n + 1 + RPW - 1) / RPW;
  P.tiles = grouped_tiles(P.wstrips, P.rgroups);
  const int blocks = fused_batch(P.B, P.tiles, 0);
  if (A.op == 0)
    hipLaunchKernelGGL((k_smooth3<0, RPW, MODE, T>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
  else if (A.op == 2)
    hipLaunchKernelGGL((k_smooth3<2, RPW, MODE, T>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
  else
    hipLaunchKernelGGL((k_smooth3<1, RPW, MODE, T>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
}

template <typename T>
void stream_smooth3_from_zero(const OpDesc& A, const T* b, T* xout, double a0, double a1,
                              double g1, double a2, double g2, hipStream_t st) {
  launch_smooth3<0, T>(A, b, xout, nullptr, a0, a1, g1, a2, g2, st);
}

template <typename T>
void stream_smooth2_resid(const OpDesc& A, const T* b, T* xout, T* r, double a0, double a1,
                          double g1, hipStream_t st) {
  launch_smooth3<1, T>(A, b, xout, r, a0, a1, g1, 0.0, 0.0, st);
}
template void stream_smooth2_resid<double>(const OpDesc&, const double*, double*, double*,
                                           double, double, double, hipStream_t);
template void stream_smooth2_resid<float>(const OpDesc&, const float*, float*, float*, double,
                                          double, double, hipStream_t);
template void stream_smooth3_from_zero<double>(const OpDesc&, const double*, double*, double,
                                               double, double, double, double, hipStream_t);
template void stream_smooth3_from_zero<float>(const OpDesc&, const float*, float*, double, double,
                                              double, double, double, hipStream_t);

// The fused last two sweeps on every streamed level (BF_NO_LAST2=1: one
// sweep per pass).
bool smooth_last2_ok(int n) {
  static const bool off = [] {
    const char* v = std::getenv("BF_NO_LAST2");
    return v && v[0] == '1';
  }();
  return !off && n >= 128;
}

template <int EP, typename T, typename TO>
int stream_smooth2(const OpDesc& A, const T* x1, const T* x0, const T* b, TO* xout,
                   const double* q, double a1, double g1, double a2, double g2,
                   double* partials, hipStream_t st) {
  // float32: 6 output rows per tile (4096^2 mixed step 19.11 ms against 19.30 with
  // 8 and 19.40 with 4); float64: 4 (a 6-row tile needs over 256 registers)
  constexpr int RPW = sizeof(T) == 4 ? 6 : 4;
  Smooth2Args<T, TO> P;
  P.A = A;
  P.x1 = x1;
  P.b = b;
  P.q = q;
  P.out = xout;
  P.partials = partials;
  P.a[0] = a1;
  P.g[0] = g1;
  P.a[1] = a2;
  P.g[1] = g2;
  P.a[2] = P.g[2] = 0.0;
  P.wstrips = (A.n + kS3Cols - 1) / kS3Cols;
  P.rgroups = (A.n + 1 + RPW - 1) / RPW;
  P.tiles = grouped_tiles(P.wstrips, P.rgroups);
  // at most kStreamMaxBlocks workgroups (wavefronts loop over tiles), which
  // bounds the partials to 2 kStreamMaxBlocks; a batch with coefficient
  // records takes its weights from them, sweeps g_batch.ia and ia + 1 (x0 is
  // then read when the first of the two sweeps is not sweep 0, whose g is zero)
  const bool records = g_batch.coef != nullptr;
  const int k0 = records ? g_batch.ia : 0;
  const int blocks = fused_batch(P.B, P.tiles, k0);
  P.x0 = (records ? k0 > 0 : g1 != 0.0) ? x0 : nullptr;
  if (A.op == 0)
    hipLaunchKernelGGL((k_smooth2<0, EP, RPW, T, TO>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
  else if (A.op == 2)
    hipLaunchKernelGGL((k_smooth2<2, EP, RPW, T, TO>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
  else
    hipLaunchKernelGGL((k_smooth2<1, EP, RPW, T, TO>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
  return blocks;
}

template <typename T>
void stream_smooth_last2(const OpDesc& A, const T* x1, const T* x0, const T* b, T* xout,
                         double a1, double g1, double a2, double g2, hipStream_t st) {
  stream_smooth2<S2_NONE, T, T>(A, x1, x0, b, xout, nullptr, a1, g1, a2, g2, nullptr, st);
}
template void stream_smooth_last2<double>(const OpDesc&, const double*, const double*,
                                          const double*, double*, double, double, double,
                                          double, hipStream_t);
template void stream_smooth_last2<float>(const OpDesc&, const float*, const float*, const float*,
                                         float*, double, double, double, double, hipStream_t);
int stream_smooth_last2_dot(const OpDesc& A, const double* x1, const double* x0, const double* b,
                            double* xout, double a1, double g1, double a2, double g2,
                            double* partials, hipStream_t st) {
  return stream_smooth2<S2_DOT, double, double>(A, x1, x0, b, xout, nullptr, a1, g1, a2, g2,
                                                partials, st);
}
int stream_smooth_last2_dot2(const OpDesc& A, const float* x1, const float* x0, const float* b,
                             double* xout, const double* q, double a1, double g1, double a2,
                             double g2, double* partials, hipStream_t st) {
  return stream_smooth2<S2_DOT2, float, double>(A, x1, x0, b, xout, q, a1, g1, a2, g2, partials,
                                                st);
}
int stream_smooth_last2_dot2_f32(const OpDesc& A, const float* x1, const float* x0,
                                 const float* b, float* xout, const double* q, double a1,
                                 double g1, double a2, double g2, double* partials,
                                 hipStream_t st) {
  return stream_smooth2<S2_DOT2, float, float>(A, x1, x0, b, xout, q, a1, g1, a2, g2, partials,
                                               st);
}

// The coarse-grid correction and the post-smoother in one pass (k_post).
// Single grids, streamed levels, sweep 0 without a momentum term; the
// Cahn-Hilliard operator with degree 2 or 3, the Laplacian with degree 2 (the
// window must start on an even fine row: D R even).  BF_NO_POST=1 switches it
// off.
bool post_ok(int n, int op, int degree, double g0, int elem_bytes) {
  static const bool off = env_int("BF_NO_POST", 0) != 0;
  // float64: the 13-point operator's three-sweep window takes 230-260
  // registers (two rows per tile), so from 2048^2 up the separate passes are
  // faster (4096^2 float64 CH V-cycle 717.7 us with this pass up to 1024^2,
  // 730.0 up to 2048^2, 805.8 up to 4096^2); the 5-point operator's window is
  // small enough at every size (Laplacian V-cycle 398.0 us with the pass on
  // every level, 430.3 up to 2048^2).  BF_POST_F64_MAX / BF_POST_F64_MAX_LAP
  // change the largest float64 level.
  static const int f64_max_ch = env_int("BF_POST_F64_MAX", 1024);
  static const int f64_max_lap = env_int("BF_POST_F64_MAX_LAP", 1 << 20);
  const BatchCtx& B = g_batch;
  const bool shape = (op == 1 && (degree == 2 || degree == 3)) || (op == 0 && degree == 2);
  const int f64_max = op == 0 ? f64_max_lap : f64_max_ch;
  return !off && shape && n >= 128 && (elem_bytes == 4 || n <= f64_max) && g0 == 0.0 &&
         B.count <= 1 && !B.coef && !B.active;
}

template <int EP, int RPW, typename T, typename TO>
static int post_launch_rpw(const OpDesc& A, int degree, const T* x, const T* e, const T* b,
                           const double* q, TO* out, const double* a, const double* g,
                           double* partials, hipStream_t st) {
  PostArgs<T, TO> P{};
  P.A = A;
  P.x = x;
  P.e = e;
  P.b = b;
  P.q = q;
  P.out = out;
  P.partials = partials;
  for (int k = 0; k < 3; ++k) {
    P.a[k] = a[k];
    P.g[k] = g[k];
  }
  const int cols = degree == 3 ? PostGeom<3>::kCols : PostGeom<2>::kCols;
  P.wstrips = (A.n + cols - 1) / cols;
  P.rgroups = (A.n + 1 + RPW - 1) / RPW;
  P.tiles = grouped_tiles(P.wstrips, P.rgroups);
  const int wpb = kStreamTPB / 64;
  const int blocks = std::min((P.tiles + wpb - 1) / wpb, kStreamMaxBlocks);
  const dim3 grid(blocks), blk(kStreamTPB);
  if (A.op == 1) {
    if (degree == 3)
      hipLaunchKernelGGL((k_post<1, 3, EP, RPW, T, TO>), grid, blk, 0, st, P);
    else
      hipLaunchKernelGGL((k_post<1, 2, EP, RPW, T, TO>), grid, blk, 0, st, P);
  } else {
    hipLaunchKernelGGL((k_post<0, 2, EP, RPW, T, TO>), grid, blk, 0, st, P);  // degree 2 only
  }
  return blocks;
}

// Tile rows: float64 2; float32 12 by default above the small levels (233
// registers for the 13-point operator; BF_POST_RPW=4, 6 or 8 selects another
// height; the window of x0 .. x2 and b lives in registers).
template <int EP, typename T, typename TO>
static int post_launch(const OpDesc& A, int degree, const T* x, const T* e, const T* b,
                       const double* q, TO* out, const double* a, const double* g,
                       double* partials, hipStream_t st) {
  if constexpr (sizeof(T) == 8) {
    return post_launch_rpw<EP, 2>(A, degree, x, e, b, q, out, a, g, partials, st);
  } else {
    static const int rpw_env = env_int("BF_POST_RPW", 12);
    const int rpw = small_level_rpw(A.n, rpw_env);
    if (rpw == 2) return post_launch_rpw<EP, 2>(A, degree, x, e, b, q, out, a, g, partials, st);
    if (rpw == 4) return post_launch_rpw<EP, 4>(A, degree, x, e, b, q, out, a, g, partials, st);
    if (rpw == 6) return post_launch_rpw<EP, 6>(A, degree, x, e, b, q, out, a, g, partials, st);
    if (rpw == 12) return post_launch_rpw<EP, 12>(A, degree, x, e, b, q, out, a, g, partials, st);
    return post_launch_rpw<EP, 8>(A, degree, x, e, b, q, out, a, g, partials, st);
  }
}

template <typename T>
void stream_post(const OpDesc& A, int degree, const T* x, const T* e, const T* b, T* out,
                 const double* a, const double* g, hipStream_t st) {
  post_launch<S2_NONE, T, T>(A, degree, x, e, b, nullptr, out, a, g, nullptr, st);
}
int stream_post_dot(const OpDesc& A, int degree, const double* x, const double* e,
                    const double* b, double* out, const double* a, const double* g,
                    double* partials, hipStream_t st) {
  return post_launch<S2_DOT, double, double>(A, degree, x, e, b, nullptr, out, a, g, partials,
                                             st);
}
// With q null only the partials of <b, z>_W (q is not read).
int stream_post_dot2(const OpDesc& A, int degree, const float* x, const float* e, const float* b,
                     double* out, const double* q, const double* a, const double* g,
                     double* partials, hipStream_t st) {
  if (!q) return post_launch<S2_DOT, float, double>(A, degree, x, e, b, q, out, a, g, partials, st);
  return post_launch<S2_DOT2, float, double>(A, degree, x, e, b, q, out, a, g, partials, st);
}
int stream_post_dot2_f32(const OpDesc& A, int degree, const float* x, const float* e,
                         const float* b, float* out, const double* q, const double* a,
                         const double* g, double* partials, hipStream_t st) {
  if (!q) return post_launch<S2_DOT, float, float>(A, degree, x, e, b, q, out, a, g, partials, st);
  return post_launch<S2_DOT2, float, float>(A, degree, x, e, b, q, out, a, g, partials, st);
}
// The coarse-grid correction and the first post-sweep in one pass (k_post
// with D = 1, 13-point operator): x1 = x0 + a0 D^{-1}(b - A x0) with
// x0 = x + P e formed on load; writes x1 and x0 (the next sweep's (x1 - x0)
// term).  For the float64 levels where the three-sweep pass does not fit the
// registers; 4-row tiles.  BF_NO_POST1=1 keeps the separate passes.
bool post1_ok(int n, int op, int degree, double g0) {
  static const bool off = env_int("BF_NO_POST1", 0) != 0;
  const BatchCtx& B = g_batch;
  return !off && op == 1 && degree == 3 && g0 == 0.0 && n >= 128 && B.count <= 1 && !B.coef &&
         !B.active;
}

template <typename T>
void stream_post1(const OpDesc& A, const T* x, const T* e, const T* b, T* x1, T* x0, double a0,
                  hipStream_t st) {
  constexpr int RPW = 4;
  PostArgs<T, T> P{};
  P.A = A;
  P.x = x;
  P.e = e;
  P.b = b;
  P.out = x1;
  P.x0out = x0;
  P.a[0] = a0;
  P.wstrips = (A.n + PostGeom<1>::kCols - 1) / PostGeom<1>::kCols;
  P.rgroups = (A.n + 1 + RPW - 1) / RPW;
  P.tiles = grouped_tiles(P.wstrips, P.rgroups);
  const int wpb = kStreamTPB / 64;
  const int blocks = std::min((P.tiles + wpb - 1) / wpb, kStreamMaxBlocks);
  hipLaunchKernelGGL((k_post<1, 1, S2_NONE, RPW, T, T>), dim3(blocks), dim3(kStreamTPB), 0, st, P);
}
template void stream_post1<double>(const OpDesc&, const double*, const double*, const double*,
                                   double*, double*, double, hipStream_t);

template void stream_post<double>(const OpDesc&, int, const double*, const double*, const double*,
                                  double*, const double*, const double*, hipStream_t);
template void stream_post<float>(const OpDesc&, int, const float*, const float*, const float*,
                                 float*, const double*, const double*, hipStream_t);

template int stream_residual<double>(const OpDesc&, const double*, const double*, double*,
                                     double*, hipStream_t);
template int stream_residual<float>(const OpDesc&, const float*, const float*, float*, double*,
                                    hipStream_t);
template void stream_smooth<double>(const OpDesc&, const double*, const double*, const double*,
                                    double*, double, double, hipStream_t);
template void stream_smooth<float>(const OpDesc&, const float*, const float*, const float*,
                                   float*, double, double, hipStream_t);
template void stream_smooth_from_zero<double>(const OpDesc&, const double*, double*, double,
                                              double, double, hipStream_t);
template void stream_smooth_from_zero<float>(const OpDesc&, const float*, float*, double, double,
                                             double, hipStream_t);
template void stream_smooth_prev_from_b<double>(const OpDesc&, const double*, const double*,
                                                double*, double, double, double, hipStream_t);
template void stream_smooth_prev_from_b<float>(const OpDesc&, const float*, const float*, float*,
                                               double, double, double, hipStream_t);

}  // namespace bf
