// Streaming stencil kernels for the large grid levels.
//
// Tiling: a block of TPB threads owns a strip of TX = 2*TPB columns (two
// adjacent columns per lane, 16-byte loads and stores) and a chunk of TY
// rows, which it walks top to bottom.  Each lane keeps the vertical window of
// its two columns (rows j-R .. j+R, R = 1 for the 5-point and 2 for the
// 13-point operator) in registers, prefetching two rows ahead; the horizontal
// neighbours come from a ring of four LDS rows (TX + 4 doubles each, the
// two-column halos on both sides loaded by lanes 0..3 with periodic wrap).
// One barrier per output row.  Ghost rows outside 0..n are the reflected rows
// of the two-layer even reflection (paper, Sec. 4, eq. discreteBC).
//
// XCD-aware launch: workgroups are dealt round-robin to the 8 XCDs of the
// MI355X, so block b runs on XCD b % 8; tiles are numbered strip-major and
// each XCD receives a contiguous range of them, so vertically adjacent
// chunks (which re-read each other's halo rows) share that XCD's L2.
#include <hip/hip_runtime.h>

#include <cstdlib>

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
};

struct StreamArgs {
  OpDesc A;
  Geo G;
  const double* x;
  const double* b;
  const double* xprev;
  double* out;
  double* partials;
  double a, g, a0;
  int ty, chunks, tiles, per_xcd;
  double* out2;        // E_CG_P: p'
  double* xu;          // E_CG_P: x (updated in place)
  const double* scal;  // E_CG_P: device scalars (alpha, beta)
  int first;           // E_CG_P: first step after a (re)start: p' = z, no x update
  int xcd_map;         // 1: deal contiguous tile ranges to the 8 XCDs
};

template <int OP, int EPI, int TPB>
__global__ void __launch_bounds__(TPB) k_stream(StreamArgs P) {
  constexpr int R = (OP == 0) ? 1 : 2;
  constexpr int W = 2 * R + 1;
  constexpr int TX = 2 * TPB;
  constexpr int LW = TX + 4;
  constexpr bool SMOOTH = (EPI == E_SMOOTH || EPI == E_SMOOTH_XB || EPI == E_SMOOTH_PB ||
                           EPI == E_SMOOTH_DOT);
  constexpr bool RED = (EPI == E_APPLY_DOT || EPI == E_RESID_NORM || EPI == E_APPLY_DOT_DD ||
                        EPI == E_RESID_DD || EPI == E_SMOOTH_DOT || EPI == E_CG_P);
  constexpr bool NEEDB = (EPI == E_RESID || EPI == E_RESID_NORM || SMOOTH || EPI == E_RESID_DD);
  __shared__ double lds[4][LW];

  const int bid = blockIdx.x;
  const int t = P.xcd_map ? (bid & 7) * P.per_xcd + (bid >> 3) : bid;
  if (t >= P.tiles) {
    if (RED && threadIdx.x == 0) {
      P.partials[bid] = 0.0;
      if (EPI == E_RESID_DD) P.partials[gridDim.x + bid] = 0.0;
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
  const int c = col0 + 2 * tid;  // own columns c, c+1
  const int lc = 2 + 2 * tid;    // their LDS index
  const bool hthread = tid < 4;
  int hcol = 0, hslot = 0;
  if (hthread) {
    hcol = (tid < 2) ? ((col0 - 2 + tid) & mask) : ((col0 + TX + tid - 2) & mask);
    hslot = (tid < 2) ? tid : (TX + tid);
  }
  const double* __restrict__ X = P.x;
  double beta = 0.0, alpha_prev = 0.0;
  if (EPI == E_CG_P && !P.first) {
    beta = P.scal[S_BETA];
    alpha_prev = P.scal[S_ALPHA];
  }

  auto dinv_row = [&](int jr) {
    return (OP == 1 && (jr == 1 || jr == n - 1)) ? P.A.dinv_edge : P.A.dinv_int;
  };
  auto load_row = [&](int jj, double2& own, double& halo) {
    const int jr = refl(jj, n);
    const double* row = X + (int64_t)jr * n;
    own = *reinterpret_cast<const double2*>(row + c);
    halo = hthread ? row[hcol] : 0.0;
    if (EPI == E_CG_P && !P.first) {
      const double* prow = P.xprev + (int64_t)jr * n;
      const double2 po = *reinterpret_cast<const double2*>(prow + c);
      own.x += beta * po.x;
      own.y += beta * po.y;
      if (hthread) halo += beta * prow[hcol];
    }
    if (EPI == E_SMOOTH_XB) {
      const double sc = P.a0 * dinv_row(jr);
      own.x *= sc;
      own.y *= sc;
      halo *= sc;
    }
  };
  auto load_ep = [&](int jj, double2& bb, double2& pp) {
    if (jj > n) return;
    const int64_t o = (int64_t)jj * n + c;
    if (NEEDB) bb = *reinterpret_cast<const double2*>(P.b + o);
    if ((EPI == E_SMOOTH || EPI == E_SMOOTH_DOT) && P.xprev)
      pp = *reinterpret_cast<const double2*>(P.xprev + o);
  };
  auto store_lds = [&](int slot, const double2& own, double halo) {
    *reinterpret_cast<double2*>(&lds[slot][lc]) = own;
    if (hthread) lds[slot][hslot] = halo;
  };

  // Sweep direction alternates with the chunk: even chunks walk down, odd
  // chunks walk up.  Two neighbouring chunks then read the rows they share
  // (the 2-row halos) in the same phase of their sweeps -- both at the start or
  // both at the end -- so the second read hits L2 instead of going out to
  // memory again.  w[k] holds row j + (k - R) * dir (dir = +-1).
  const int dir = (chunk & 1) ? -1 : 1;
  const int len = j1 - j0;
  const int jstart = dir > 0 ? j0 : j1 - 1;
  double2 w[W];
  double hw[W];
#pragma unroll
  for (int k = 0; k < W; ++k) load_row(jstart + (k - R) * dir, w[k], hw[k]);
  // prefetch queue: the rows entering the window at steps s+1 and s+2; rows
  // beyond the tile's last need are never loaded
  double2 q0 = make_double2(0.0, 0.0), q1 = make_double2(0.0, 0.0);
  double hq0 = 0.0, hq1 = 0.0;
  if (1 < len) load_row(jstart + (R + 1) * dir, q0, hq0);
  if (2 < len) load_row(jstart + (R + 2) * dir, q1, hq1);
  double2 bq = make_double2(0.0, 0.0), pq = make_double2(0.0, 0.0);
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
    const double2 bcur = bq, pcur = pq;
    if (s + 1 < len) load_ep(j + dir, bq, pq);

    // rows j-1 / j+1 (and j-2 / j+2) in the window, whatever the direction
    const double2 wm1 = dir > 0 ? w[R - 1] : w[R + 1];
    const double2 wp1 = dir > 0 ? w[R + 1] : w[R - 1];
    const double* L0 = lds[j & 3];
    const double2 cl = *reinterpret_cast<const double2*>(&L0[lc - 2]);  // c-2, c-1
    const double2 cr = *reinterpret_cast<const double2*>(&L0[lc + 2]);  // c+2, c+3
    Nb13 v0, v1;
    v0.c = w[R].x;
    v1.c = w[R].y;
    v0.xm1 = cl.y;
    v0.xp1 = w[R].y;
    v1.xm1 = w[R].x;
    v1.xp1 = cr.x;
    v0.ym1 = wm1.x;
    v0.yp1 = wp1.x;
    v1.ym1 = wm1.y;
    v1.yp1 = wp1.y;
    if (R == 2) {
      const double2 wm2 = dir > 0 ? w[0] : w[W - 1];
      const double2 wp2 = dir > 0 ? w[W - 1] : w[0];
      const double* Lm = lds[(j - 1) & 3];
      const double* Lp = lds[(j + 1) & 3];
      v0.xm2 = cl.x;
      v0.xp2 = cr.x;
      v1.xm2 = cl.y;
      v1.xp2 = cr.y;
      v0.ym2 = wm2.x;
      v0.yp2 = wp2.x;
      v1.ym2 = wm2.y;
      v1.yp2 = wp2.y;
      v0.dmm = Lm[lc - 1];
      v0.dmp = wm1.y;
      v1.dmm = wm1.x;
      v1.dmp = Lm[lc + 2];
      v0.dpm = Lp[lc - 1];
      v0.dpp = wp1.y;
      v1.dpm = wp1.x;
      v1.dpp = Lp[lc + 2];
    }
    const int64_t o = (int64_t)j * n + c;
    const double wgt = row_weight(j, n);
    double2 res;
    if (EPI == E_APPLY || EPI == E_APPLY_DOT) {
      res.x = apply_vals<OP>(v0, P.A.coef);
      res.y = apply_vals<OP>(v1, P.A.coef);
      if (EPI == E_APPLY_DOT) acc += wgt * (v0.c * res.x + v1.c * res.y);
    } else if (EPI == E_RESID || EPI == E_RESID_NORM) {
      res.x = bcur.x - apply_vals<OP>(v0, P.A.coef);
      res.y = bcur.y - apply_vals<OP>(v1, P.A.coef);
      if (EPI == E_RESID_NORM) acc += wgt * (res.x * res.x + res.y * res.y);
    } else if (SMOOTH) {
      const double dinv = dinv_row(j);
      const double ad = P.a * dinv;
      double2 prev = make_double2(0.0, 0.0);
      if (EPI == E_SMOOTH_PB) {
        prev.x = P.a0 * dinv * bcur.x;
        prev.y = P.a0 * dinv * bcur.y;
      } else if (EPI != E_SMOOTH_XB && P.xprev) {
        prev = pcur;
      }
      res.x = v0.c + ad * (bcur.x - apply_vals<OP>(v0, P.A.coef)) + P.g * (v0.c - prev.x);
      res.y = v1.c + ad * (bcur.y - apply_vals<OP>(v1, P.A.coef)) + P.g * (v1.c - prev.y);
      if (EPI == E_SMOOTH_DOT) acc += wgt * (bcur.x * res.x + bcur.y * res.y);
    } else if (EPI == E_APPLY_DOT_DD) {
      res.x = -residual_dd_vals<OP>(v0, 0.0, P.A.coef);
      res.y = -residual_dd_vals<OP>(v1, 0.0, P.A.coef);
      acc += wgt * (v0.c * res.x + v1.c * res.y);
    } else if (EPI == E_CG_P) {
      if (OP == 1) {
        res.x = -residual_dd_vals<OP>(v0, 0.0, P.A.coef);
        res.y = -residual_dd_vals<OP>(v1, 0.0, P.A.coef);
      } else {
        res.x = apply_vals<OP>(v0, P.A.coef);
        res.y = apply_vals<OP>(v1, P.A.coef);
      }
      acc += wgt * (v0.c * res.x + v1.c * res.y);
      *reinterpret_cast<double2*>(P.out2 + o) = make_double2(v0.c, v1.c);
      if (!P.first) {
        const double2 po = *reinterpret_cast<const double2*>(P.xprev + o);
        double2 xv = *reinterpret_cast<const double2*>(P.xu + o);
        xv.x += alpha_prev * po.x;
        xv.y += alpha_prev * po.y;
        *reinterpret_cast<double2*>(P.xu + o) = xv;
      }
    } else {  // E_RESID_DD
      res.x = residual_dd_vals<OP>(v0, bcur.x, P.A.coef);
      res.y = residual_dd_vals<OP>(v1, bcur.y, P.A.coef);
      acc += wgt * (res.x * res.x + res.y * res.y);
      const double u0 = ulp_of(v0.c), u1 = ulp_of(v1.c);
      acc2 += wgt * (u0 * u0 + u1 * u1);
    }
    *reinterpret_cast<double2*>(P.out + o) = res;

#pragma unroll
    for (int k = 0; k < W - 1; ++k) {
      w[k] = w[k + 1];
      hw[k] = hw[k + 1];
    }
    w[W - 1] = q0;
    hw[W - 1] = hq0;
    q0 = q1;
    hq0 = hq1;
    if (s + 3 < len) load_row(j + (R + 3) * dir, q1, hq1);
  }
  if (RED) {
    const double s = block_sum_n<TPB>(acc);
    if (tid == 0) P.partials[bid] = s;
    if (EPI == E_RESID_DD) {
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

bool stream_ok(int n) { return n >= 128; }

StreamCfg stream_cfg(int n) {
  StreamCfg c;
  c.tpb = n >= 1024 ? 256 : (n >= 256 ? 128 : 64);
  const int tx = 2 * c.tpb;
  const int strips = n / tx;
  // aim at ~4096 tiles (16 per CU over the 256 CUs), 8..64 rows each; on
  // 4096^2 this gives 8-row tiles, measured fastest for whole solves
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

template <int OP, int EPI>
static void dispatch(const StreamCfg& c, const StreamArgs& P, hipStream_t st) {
  switch (c.tpb) {
    case 256:
      hipLaunchKernelGGL((k_stream<OP, EPI, 256>), dim3(c.blocks), dim3(256), 0, st, P);
      break;
    case 128:
      hipLaunchKernelGGL((k_stream<OP, EPI, 128>), dim3(c.blocks), dim3(128), 0, st, P);
      break;
    default:
      hipLaunchKernelGGL((k_stream<OP, EPI, 64>), dim3(c.blocks), dim3(64), 0, st, P);
      break;
  }
}

template <int EPI>
static int stream_launch(const OpDesc& A, const double* x, const double* b, const double* xprev,
                         double* out, double* partials, double a, double g, hipStream_t st,
                         double a0 = 0.0) {
  const StreamCfg c = stream_cfg(A.n);
  StreamArgs P{};
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
  return stream_launch<E_APPLY>(A, x, nullptr, nullptr, y, nullptr, 0, 0, st);
}
int stream_apply_dot(const OpDesc& A, const double* p, double* q, double* partials, bool dd,
                     hipStream_t st) {
  if (dd) return stream_launch<E_APPLY_DOT_DD>(A, p, nullptr, nullptr, q, partials, 0, 0, st);
  return stream_launch<E_APPLY_DOT>(A, p, nullptr, nullptr, q, partials, 0, 0, st);
}
int stream_residual(const OpDesc& A, const double* x, const double* b, double* r,
                    double* partials, hipStream_t st) {
  if (partials) return stream_launch<E_RESID_NORM>(A, x, b, nullptr, r, partials, 0, 0, st);
  return stream_launch<E_RESID>(A, x, b, nullptr, r, nullptr, 0, 0, st);
}
int stream_residual_dd(const OpDesc& A, const double* x, const double* b, double* r,
                       double* partials, hipStream_t st) {
  return stream_launch<E_RESID_DD>(A, x, b, nullptr, r, partials, 0, 0, st);
}
void stream_smooth(const OpDesc& A, const double* x, const double* xprev, const double* b,
                   double* xout, double a, double g, hipStream_t st) {
  stream_launch<E_SMOOTH>(A, x, b, xprev, xout, nullptr, a, g, st);
}
void stream_smooth_from_zero(const OpDesc& A, const double* b, double* xout, double a0, double a1,
                             double g1, hipStream_t st) {
  stream_launch<E_SMOOTH_XB>(A, b, b, nullptr, xout, nullptr, a1, g1, st, a0);
}
void stream_smooth_prev_from_b(const OpDesc& A, const double* x, const double* b, double* xout,
                               double a0, double a, double g, hipStream_t st) {
  stream_launch<E_SMOOTH_PB>(A, x, b, nullptr, xout, nullptr, a, g, st, a0);
}
int stream_smooth_dot(const OpDesc& A, const double* x, const double* xprev, const double* b,
                      double* xout, double a, double g, double* partials, hipStream_t st) {
  return stream_launch<E_SMOOTH_DOT>(A, x, b, xprev, xout, partials, a, g, st);
}
int stream_cg_p(const OpDesc& A, const double* z, const double* p_old, double* p_new, double* q,
                double* x, const double* scal, bool first, double* partials, hipStream_t st) {
  const StreamCfg c = stream_cfg(A.n);
  StreamArgs P{};
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

}  // namespace bf
