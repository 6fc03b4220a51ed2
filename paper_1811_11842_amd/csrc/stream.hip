// Streaming stencil kernels for the large grid levels.
//
// Tiling: a block of TPB threads owns a strip of TX = V*TPB columns (V
// adjacent columns per lane, 16-byte loads and stores: V = 2 for float64,
// 4 for float32) and a chunk of TY rows, which it walks row by row.  Each
// lane keeps the vertical window of its columns (rows j-R .. j+R, R = 1 for
// the 5-point and 2 for the 13-point operator) in registers, prefetching two
// rows ahead; the horizontal neighbours come from a ring of four LDS rows
// (TX + 4 values each, the two-column halos on both sides loaded by lanes
// 0..3 with periodic wrap).  One barrier per output row.  Ghost rows outside
// 0..n are the reflected rows of the two-layer even reflection (paper,
// Sec. 4, eq. discreteBC).
//
// Sweep direction alternates with the chunk (even chunks walk down, odd
// chunks walk up), so two neighbouring chunks read the rows they share in the
// same phase of their sweeps and the second read is served by L2.
//
// XCD-aware launch: workgroups are dealt round-robin to the 8 XCDs of the
// MI355X, so block b runs on XCD b % 8; tiles are numbered strip-major and
// each XCD receives a contiguous range of them.
#include <hip/hip_runtime.h>

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
  E_SMOOTH_DOT2 = 11   // E_SMOOTH and partials of <b, out>_W and <out, q>_W (q float64)
};

// 16-byte vector of V elements of T, and a pair for the LDS halo reads.
template <typename T, int V>
struct alignas(16) VecN {
  T v[V];
};
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T v[2];
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
  int ty, chunks, tiles, per_xcd;
  double* out2;        // E_CG_P: p'
  double* xu;          // E_CG_P: x (updated in place)
  const double* scal;  // E_CG_P: device scalars (alpha, beta)
  const double* q;     // E_SMOOTH_DOT2: second vector of the extra dot
  int first;           // E_CG_P: first step after a (re)start: p' = z, no x update
  int xcd_map;         // 1: deal contiguous tile ranges to the 8 XCDs
};

template <int OP, int EPI, int TPB, typename T, typename TO>
__global__ void __launch_bounds__(TPB) k_stream(StreamArgs<T, TO> P) {
  constexpr int V = 16 / sizeof(T);
  constexpr int R = (OP == 0) ? 1 : 2;
  constexpr int W = 2 * R + 1;
  constexpr int TX = V * TPB;
  constexpr int LW = TX + 4;
  constexpr bool SMOOTH = (EPI == E_SMOOTH || EPI == E_SMOOTH_XB || EPI == E_SMOOTH_PB ||
                           EPI == E_SMOOTH_DOT || EPI == E_SMOOTH_DOT2);
  constexpr bool RED = (EPI == E_APPLY_DOT || EPI == E_RESID_NORM || EPI == E_APPLY_DOT_DD ||
                        EPI == E_RESID_DD || EPI == E_SMOOTH_DOT || EPI == E_CG_P ||
                        EPI == E_SMOOTH_DOT2);
  constexpr bool RED2 = (EPI == E_RESID_DD || EPI == E_SMOOTH_DOT2);
  constexpr bool NEEDB = (EPI == E_RESID || EPI == E_RESID_NORM || SMOOTH || EPI == E_RESID_DD);
  constexpr bool NEEDP = (EPI == E_SMOOTH || EPI == E_SMOOTH_DOT || EPI == E_SMOOTH_DOT2);
  using VT = VecN<T, V>;
  using VO = VecN<TO, V>;
  __shared__ T lds[4][LW];

  const int bid = blockIdx.x;
  const int t = P.xcd_map ? (bid & 7) * P.per_xcd + (bid >> 3) : bid;
  if (t >= P.tiles) {
    if (RED && threadIdx.x == 0) {
      P.partials[bid] = 0.0;
      if (RED2) P.partials[gridDim.x + bid] = 0.0;
    }
    return;
  }
  const int n = P.G.n, mask = P.G.mask;
  const int strip = t / P.chunks;
  const int chunk = t - strip * P.chunks;
  const int j0 = chunk * P.ty;
  const int j1 = min(j0 + P.ty, n + 1);
  const int col0 = strip * TX;
  const int tid = threadIdx.x;
  const int c = col0 + V * tid;  // own columns c .. c+V-1
  const int lc = 2 + V * tid;    // their LDS index
  const bool hthread = tid < 4;
  int hcol = 0, hslot = 0;
  if (hthread) {
    hcol = (tid < 2) ? ((col0 - 2 + tid) & mask) : ((col0 + TX + tid - 2) & mask);
    hslot = (tid < 2) ? tid : (TX + tid);
  }
  const T* __restrict__ X = P.x;
  const T coef = T(P.A.coef);
  const T ca = T(P.a), cg = T(P.g), ca0 = T(P.a0);
  double beta = 0.0, alpha_prev = 0.0;
  if constexpr (EPI == E_CG_P) {
    if (!P.first) {
      beta = P.scal[S_BETA];
      alpha_prev = P.scal[S_ALPHA];
    }
  }

  auto dinv_row = [&](int jr) -> T {
    return T((OP == 1 && (jr == 1 || jr == n - 1)) ? P.A.dinv_edge : P.A.dinv_int);
  };
  auto load_row = [&](int jj, T(&own)[V], T& halo) {
    const int jr = refl(jj, n);
    const T* row = X + (int64_t)jr * n;
    const VT v = *reinterpret_cast<const VT*>(row + c);
#pragma unroll
    for (int i = 0; i < V; ++i) own[i] = v.v[i];
    halo = hthread ? row[hcol] : T(0);
    if constexpr (EPI == E_CG_P) {
      if (!P.first) {
        const T* prow = P.xprev + (int64_t)jr * n;
        const VT po = *reinterpret_cast<const VT*>(prow + c);
#pragma unroll
        for (int i = 0; i < V; ++i) own[i] += beta * po.v[i];
        if (hthread) halo += beta * prow[hcol];
      }
    }
    if constexpr (EPI == E_SMOOTH_XB) {
      const T sc = ca0 * dinv_row(jr);
#pragma unroll
      for (int i = 0; i < V; ++i) own[i] *= sc;
      halo *= sc;
    }
  };
  auto load_ep = [&](int jj, VT& bb, VT& pp) {
    if (jj > n) return;
    const int64_t o = (int64_t)jj * n + c;
    if (NEEDB) bb = *reinterpret_cast<const VT*>(P.b + o);
    if (NEEDP && P.xprev) pp = *reinterpret_cast<const VT*>(P.xprev + o);
  };
  auto store_lds = [&](int slot, const T(&own)[V], T halo) {
    VT v;
#pragma unroll
    for (int i = 0; i < V; ++i) v.v[i] = own[i];
    *reinterpret_cast<VT*>(&lds[slot][lc]) = v;
    if (hthread) lds[slot][hslot] = halo;
  };

  // w[k] holds row j + (k - R) * dir of the lane's columns (dir = +-1).
  const int dir = (chunk & 1) ? -1 : 1;
  const int len = j1 - j0;
  const int jstart = dir > 0 ? j0 : j1 - 1;
  T w[W][V];
  T hw[W];
#pragma unroll
  for (int k = 0; k < W; ++k) load_row(jstart + (k - R) * dir, w[k], hw[k]);
  // prefetch queue: the rows entering the window at steps s+1 and s+2; rows
  // beyond the tile's last need are never loaded
  T q0[V], q1[V];
  T hq0 = T(0), hq1 = T(0);
#pragma unroll
  for (int i = 0; i < V; ++i) q0[i] = q1[i] = T(0);
  if (1 < len) load_row(jstart + (R + 1) * dir, q0, hq0);
  if (2 < len) load_row(jstart + (R + 2) * dir, q1, hq1);
  VT bq{}, pq{};
  load_ep(jstart, bq, pq);
  if (R == 2) {
    store_lds((jstart - dir) & 3, w[1], hw[1]);
    store_lds(jstart & 3, w[2], hw[2]);
  }

  double acc = 0.0, acc2 = 0.0;
  for (int s = 0; s < len; ++s) {
    const int j = jstart + s * dir;
    if (R == 2)
      store_lds((j + dir) & 3, w[3], hw[3]);
    else
      store_lds(j & 3, w[1], hw[1]);
    __syncthreads();
    const VT bcur = bq, pcur = pq;
    if (s + 1 < len) load_ep(j + dir, bq, pq);

    // rows of the window by their true offset from j, whatever the direction
    const T* wm1 = dir > 0 ? w[R - 1] : w[R + 1];
    const T* wp1 = dir > 0 ? w[R + 1] : w[R - 1];
    const T* L0 = lds[j & 3];
    // rowj: columns c-2 .. c+V+1 of row j
    T rowj[V + 4];
    {
      const Pair<T> l = *reinterpret_cast<const Pair<T>*>(&L0[lc - 2]);
      const Pair<T> r = *reinterpret_cast<const Pair<T>*>(&L0[lc + V]);
      rowj[0] = l.v[0];
      rowj[1] = l.v[1];
#pragma unroll
      for (int i = 0; i < V; ++i) rowj[2 + i] = w[R][i];
      rowj[V + 2] = r.v[0];
      rowj[V + 3] = r.v[1];
    }
    Nb13T<T> nb[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      nb[i].c = rowj[i + 2];
      nb[i].xm1 = rowj[i + 1];
      nb[i].xp1 = rowj[i + 3];
      nb[i].ym1 = wm1[i];
      nb[i].yp1 = wp1[i];
    }
    if (R == 2) {
      const T* wm2 = dir > 0 ? w[0] : w[W - 1];
      const T* wp2 = dir > 0 ? w[W - 1] : w[0];
      const T* Lm = lds[(j - 1) & 3];
      const T* Lp = lds[(j + 1) & 3];
      T rowm[V + 2], rowp[V + 2];
      rowm[0] = Lm[lc - 1];
      rowm[V + 1] = Lm[lc + V];
      rowp[0] = Lp[lc - 1];
      rowp[V + 1] = Lp[lc + V];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        rowm[1 + i] = wm1[i];
        rowp[1 + i] = wp1[i];
      }
#pragma unroll
      for (int i = 0; i < V; ++i) {
        nb[i].xm2 = rowj[i];
        nb[i].xp2 = rowj[i + 4];
        nb[i].ym2 = wm2[i];
        nb[i].yp2 = wp2[i];
        nb[i].dmm = rowm[i];
        nb[i].dmp = rowm[i + 2];
        nb[i].dpm = rowp[i];
        nb[i].dpp = rowp[i + 2];
      }
    }
    const int64_t o = (int64_t)j * n + c;
    const double wgt = row_weight(j, n);
    VO res;
    if constexpr (EPI == E_APPLY || EPI == E_APPLY_DOT) {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const T ax = apply_vals<OP>(nb[i], coef);
        res.v[i] = TO(ax);
        if (EPI == E_APPLY_DOT) acc += wgt * double(nb[i].c) * double(ax);
      }
    } else if constexpr (EPI == E_RESID || EPI == E_RESID_NORM) {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const T r = bcur.v[i] - apply_vals<OP>(nb[i], coef);
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
        else if (EPI != E_SMOOTH_XB && P.xprev)
          prev = pcur.v[i];
        const T xn =
            nb[i].c + ad * (bcur.v[i] - apply_vals<OP>(nb[i], coef)) + cg * (nb[i].c - prev);
        res.v[i] = TO(xn);
        if (EPI == E_SMOOTH_DOT || EPI == E_SMOOTH_DOT2)
          acc += wgt * double(bcur.v[i]) * double(TO(xn));
      }
      if constexpr (EPI == E_SMOOTH_DOT2) {
        const VecN<double, V> qv = *reinterpret_cast<const VecN<double, V>*>(P.q + o);
#pragma unroll
        for (int i = 0; i < V; ++i) acc2 += wgt * double(res.v[i]) * qv.v[i];
      }
    } else if constexpr (std::is_same<T, double>::value) {
      if constexpr (EPI == E_APPLY_DOT_DD) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
          res.v[i] = -residual_dd_vals<OP>(nb[i], 0.0, P.A.coef);
          acc += wgt * nb[i].c * res.v[i];
        }
      } else if constexpr (EPI == E_CG_P) {
        VecN<double, V> pn;
#pragma unroll
        for (int i = 0; i < V; ++i) {
          res.v[i] = OP == 1 ? -residual_dd_vals<OP>(nb[i], 0.0, P.A.coef)
                             : apply_vals<OP>(nb[i], P.A.coef);
          acc += wgt * nb[i].c * res.v[i];
          pn.v[i] = nb[i].c;
        }
        *reinterpret_cast<VecN<double, V>*>(P.out2 + o) = pn;
        if (!P.first) {
          const VecN<double, V> po = *reinterpret_cast<const VecN<double, V>*>(P.xprev + o);
          VecN<double, V> xv = *reinterpret_cast<const VecN<double, V>*>(P.xu + o);
#pragma unroll
          for (int i = 0; i < V; ++i) xv.v[i] += alpha_prev * po.v[i];
          *reinterpret_cast<VecN<double, V>*>(P.xu + o) = xv;
        }
      } else if constexpr (EPI == E_RESID_DD) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
          res.v[i] = residual_dd_vals<OP>(nb[i], bcur.v[i], P.A.coef);
          acc += wgt * res.v[i] * res.v[i];
          const double u = ulp_of(nb[i].c);
          acc2 += wgt * u * u;
        }
      }
    }
    *reinterpret_cast<VO*>(P.out + o) = res;

#pragma unroll
    for (int k = 0; k < W - 1; ++k) {
#pragma unroll
      for (int i = 0; i < V; ++i) w[k][i] = w[k + 1][i];
      hw[k] = hw[k + 1];
    }
#pragma unroll
    for (int i = 0; i < V; ++i) {
      w[W - 1][i] = q0[i];
      q0[i] = q1[i];
    }
    hw[W - 1] = hq0;
    hq0 = hq1;
    if (s + 3 < len) load_row(j + (R + 3) * dir, q1, hq1);
  }
  if (RED) {
    const double s = block_sum_n<TPB>(acc);
    if (tid == 0) P.partials[bid] = s;
    if (RED2) {
      const double s2 = block_sum_n<TPB>(acc2);
      if (tid == 0) P.partials[gridDim.x + bid] = s2;
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

bool stream_ok(int n, int elem_bytes) { return n >= 64 * (16 / elem_bytes); }

StreamCfg stream_cfg(int n, int elem_bytes) {
  StreamCfg c;
  const int vcols = 16 / elem_bytes;
  c.tpb = n >= 256 * vcols ? 256 : (n >= 128 * vcols ? 128 : 64);
  const int tx = vcols * c.tpb;
  const int strips = n / tx;
  // aim at ~4096 tiles (16 per CU over the 256 CUs), 8..64 rows each; on
  // 4096^2 in float64 this gives 8-row tiles, measured fastest for whole solves
  int ty = (int)(((int64_t)(n + 1) * strips) / 4096);
  static const int ty_env = env_int("BF_STREAM_TY", 0);
  if (ty_env > 0) ty = ty_env;
  ty = ty < 8 ? 8 : (ty > 64 ? 64 : ty);
  c.ty = ty;
  c.chunks = (n + 1 + ty - 1) / ty;
  c.tiles = strips * c.chunks;
  static const int xm = env_int("BF_XCD_MAP", 1);
  c.xcd_map = xm;
  c.per_xcd = (c.tiles + 7) / 8;
  c.blocks = xm ? 8 * c.per_xcd : c.tiles;
  return c;
}

bool stream_ok(int n) { return stream_ok(n, 8); }
StreamCfg stream_cfg(int n) { return stream_cfg(n, 8); }

template <int OP, int EPI, typename T, typename TO>
static void dispatch(const StreamCfg& c, const StreamArgs<T, TO>& P, hipStream_t st) {
  switch (c.tpb) {
    case 256:
      hipLaunchKernelGGL((k_stream<OP, EPI, 256, T, TO>), dim3(c.blocks), dim3(256), 0, st, P);
      break;
    case 128:
      hipLaunchKernelGGL((k_stream<OP, EPI, 128, T, TO>), dim3(c.blocks), dim3(128), 0, st, P);
      break;
    default:
      hipLaunchKernelGGL((k_stream<OP, EPI, 64, T, TO>), dim3(c.blocks), dim3(64), 0, st, P);
      break;
  }
}

template <int EPI, typename T, typename TO>
static int stream_launch(const OpDesc& A, const T* x, const T* b, const T* xprev, TO* out,
                         double* partials, double a, double g, hipStream_t st, double a0 = 0.0,
                         const double* q = nullptr) {
  const StreamCfg c = stream_cfg(A.n, sizeof(T));
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
  P.ty = c.ty;
  P.chunks = c.chunks;
  P.tiles = c.tiles;
  P.per_xcd = c.per_xcd;
  P.xcd_map = c.xcd_map;
  if (A.op == 0)
    dispatch<0, EPI>(c, P, st);
  else
    dispatch<1, EPI>(c, P, st);
  return c.blocks;
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
                       double* partials, hipStream_t st) {
  return stream_launch<E_RESID_DD, double, double>(A, x, b, nullptr, r, partials, 0, 0, st);
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
int stream_cg_p(const OpDesc& A, const double* z, const double* p_old, double* p_new, double* q,
                double* x, const double* scal, bool first, double* partials, hipStream_t st) {
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
  P.ty = c.ty;
  P.chunks = c.chunks;
  P.tiles = c.tiles;
  P.per_xcd = c.per_xcd;
  P.xcd_map = c.xcd_map;
  if (A.op == 0)
    dispatch<0, E_CG_P>(c, P, st);
  else
    dispatch<1, E_CG_P>(c, P, st);
  return c.blocks;
}

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
