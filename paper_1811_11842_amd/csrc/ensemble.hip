// Ensemble driver: many independent instances of the step, of uneven sizes
// and with their own parameters, advanced together.
//
// Instances are grouped by grid size into classes.  A class of B instances
// of size n stores every field as one array of B consecutive (n+1) x n
// blocks, and every operation on the class -- the stencil sweeps, grid
// transfers, coarse tail, Krylov updates and reductions -- is ONE launch over
// all its instances (the kernels take the instance from the workgroup index,
// see BatchCtx), with per-instance operator and smoothing coefficients and a
// per-instance convergence mask: an instance that has converged is skipped
// by the stencil kernels and its scalars are frozen while the others
// iterate.  The V-cycle of a class is captured once per operator as a HIP
// graph and replayed.  Classes run concurrently, each on its own stream and
// host thread.
//
// The solver per instance is the float64 MG-preconditioned CG of the single
// grid (double-double q = A p for the Cahn-Hilliard operator, constant-mode
// correction, double-double true residual and float64 floor estimate); it
// stops at the recursive residual and reports OK / AT_FLOOR /
// NOT_CONVERGED from the true residual, without refinement restarts.
//
// Tile height of the stencil kernels: chosen per class at creation by
// timing the smoothing sweep of that class with 4-, 5- and 8-row tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstddef>
#include <string>
#include <thread>
#include <vector>

#include "../../include/biofilm.h"
#include "common.hpp"
#include "host.hpp"
#include "kernels.hpp"

using namespace bf;

namespace {

#define EGRID(idx, total)                                                              \
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (total); \
       idx += (int64_t)gridDim.x * blockDim.x)

// Per-instance step parameters on the device.
struct EParam {
  double dtMn2, inv_npoly, chi, lo, hi;  // Flory-Huggins right-hand side
  double div_scale, vel_scale;           // n / (2 dt), dt n / 2
};

__global__ void __launch_bounds__(kBlock) ke_divergence(Geo G, int64_t stride, const EParam* prm,
                                                        const double* __restrict__ u,
                                                        const double* __restrict__ v,
                                                        double* __restrict__ rhs) {
  const int inst = blockIdx.y;
  const double scale = prm[inst].div_scale;
  u += inst * stride;
  v += inst * stride;
  rhs += inst * stride;
  EGRID(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    const int n = G.n;
    const double* ur = u + (int64_t)j * n;
    const double vp = (j == n) ? -v[(int64_t)(n - 1) * n + i] : v[idx + n];
    const double vm = (j == 0) ? -v[(int64_t)n + i] : v[idx - n];
    rhs[idx] = ((ur[(i + 1) & G.mask] - ur[(i - 1) & G.mask]) + (vp - vm)) * scale;
  }
}

__global__ void __launch_bounds__(kBlock) ke_velocity(Geo G, int64_t stride, const EParam* prm,
                                                      const double* __restrict__ p,
                                                      const double* us, const double* vs,
                                                      double* u, double* v) {
  const int inst = blockIdx.y;
  const double scale = prm[inst].vel_scale;
  const int64_t o = inst * stride;
  EGRID(idx, G.npts) {
    const int i = (int)(idx & G.mask), j = (int)(idx >> G.log2n);
    const int n = G.n;
    const double* pr = p + o + (int64_t)j * n;
    const double gx = pr[(i + 1) & G.mask] - pr[(i - 1) & G.mask];
    const double gy = p[o + (int64_t)refl(j + 1, n) * n + i] - p[o + (int64_t)refl(j - 1, n) * n + i];
    u[o + idx] = us[o + idx] - scale * gx;
    v[o + idx] = vs[o + idx] - scale * gy;
  }
}

// partials[inst * gridDim.x + block] of sum_W x y (y == nullptr: y = 1) or,
// with diff, of sum_W (x - y).
__global__ void __launch_bounds__(kBlock) ke_dot(Geo G, int64_t stride, const double* __restrict__ x,
                                                 const double* __restrict__ y, int diff,
                                                 double* __restrict__ partials) {
  const int inst = blockIdx.y;
  x += inst * stride;
  if (y) y += inst * stride;
  double acc = 0.0;
  EGRID(idx, G.npts) {
    const int j = (int)(idx >> G.log2n);
    const double yv = y ? y[idx] : 1.0;
    acc += row_weight(j, G.n) * (diff ? x[idx] - yv : x[idx] * yv);
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[inst * gridDim.x + blockIdx.x] = t;
}

// One workgroup per instance: reduce its np partials (starting at
// partials + base + inst * np) and update its scalars (modes of FinalizeMode).
__global__ void __launch_bounds__(kBlock) ke_finalize(const double* __restrict__ partials,
                                                      int64_t base, int np,
                                                      double* __restrict__ scal, int mode,
                                                      int slot, double nn,
                                                      const int* __restrict__ active) {
  const int inst = blockIdx.x;
  if (active && !active[inst]) return;
  const double* pp = partials + base + (int64_t)inst * np;
  double acc = 0.0;
  for (int k = threadIdx.x; k < np; k += kBlock) acc += pp[k];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) {
    double* sc = scal + (int64_t)inst * kNumSlots;
    switch (mode) {
      case F_STORE:
        sc[slot] = s;
        break;
      case F_ALPHA:
        sc[S_PQ] = s;
        sc[S_ALPHA] = sc[S_RZ] / s;
        break;
      case F_BETA: {
        const double old = sc[S_RZ];
        sc[S_RZOLD] = old;
        sc[S_RZ] = s;
        sc[S_BETA] = s / old;
        break;
      }
      case F_MEAN:
        sc[S_MEAN] = s / nn;
        break;
    }
  }
}

// r -= alpha q per instance, partials of ||r||_W^2 (active instances only).
__global__ void __launch_bounds__(kBlock) ke_r_update(Geo G, int64_t stride, double* __restrict__ r,
                                                      const double* __restrict__ q,
                                                      const double* __restrict__ scal,
                                                      const int* __restrict__ active,
                                                      double* __restrict__ partials) {
  const int inst = blockIdx.y;
  double acc = 0.0;
  if (!active || active[inst]) {
    const double alpha = scal[(int64_t)inst * kNumSlots + S_ALPHA];
    r += inst * stride;
    q += inst * stride;
    EGRID(idx, G.npts) {
      const int j = (int)(idx >> G.log2n);
      const double v = r[idx] - alpha * q[idx];
      r[idx] = v;
      acc += row_weight(j, G.n) * v * v;
    }
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[inst * gridDim.x + blockIdx.x] = t;
}

// Convergence of every instance after an iteration's r update, on the device
// (one workgroup): an active instance counts the iteration, keeps its
// relative recursive residual, and leaves the mask when that meets rtol (or
// is not finite), recording which p buffer holds its last direction; flags
// receive the number still active and whether a norm was not finite, for the
// host to read while the next preconditioner application runs.
__global__ void __launch_bounds__(kBlock) ke_converge(const double* __restrict__ scal,
                                                      const double* __restrict__ bn, double rtol,
                                                      int* __restrict__ active,
                                                      int* __restrict__ iters,
                                                      int* __restrict__ parity, int parity_now,
                                                      double* __restrict__ rel_res,
                                                      int* __restrict__ flags, int count) {
  int rem = 0, bad = 0;
  for (int k = threadIdx.x; k < count; k += kBlock) {
    if (!active[k]) continue;
    const double rr = scal[(int64_t)k * kNumSlots + S_RR];
    const double rel = sqrt(rr) / bn[k];
    iters[k] += 1;
    rel_res[k] = rel;
    if (!isfinite(rel)) {
      bad = 1;
      active[k] = 0;
      parity[k] = parity_now;
    } else if (rel <= rtol) {
      active[k] = 0;
      parity[k] = parity_now;
    } else {
      ++rem;
    }
  }
  const double r = block_sum((double)rem);
  const double b = block_sum((double)bad);
  if (threadIdx.x == 0) {
    flags[0] = (int)r;
    flags[1] = b > 0.0 ? 1 : 0;
  }
}

// x += alpha p for the instances with sel[inst] != 0.
__global__ void __launch_bounds__(kBlock) ke_x_update(Geo G, int64_t stride, double* __restrict__ x,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ scal,
                                                      const int* __restrict__ sel) {
  const int inst = blockIdx.y;
  if (!sel[inst]) return;
  const double alpha = scal[(int64_t)inst * kNumSlots + S_ALPHA];
  x += inst * stride;
  p += inst * stride;
  EGRID(idx, G.npts) x[idx] += alpha * p[idx];
}

// x *= scal[S_GAMMA] of the instance.
__global__ void __launch_bounds__(kBlock) ke_scale(Geo G, int64_t stride, double* __restrict__ x,
                                                   const double* __restrict__ scal) {
  const int inst = blockIdx.y;
  const double g = scal[(int64_t)inst * kNumSlots + S_GAMMA];
  x += inst * stride;
  EGRID(idx, G.npts) x[idx] *= g;
}

// y = x + sign * mean (mean = scal[S_MEAN] of the instance).
__global__ void __launch_bounds__(kBlock) ke_add_mean(Geo G, int64_t stride, const double* x,
                                                      double* y, const double* __restrict__ scal,
                                                      double sign, const int* __restrict__ sel) {
  const int inst = blockIdx.y;
  if (sel && !sel[inst]) return;
  const double m = sign * scal[(int64_t)inst * kNumSlots + S_MEAN];
  x += inst * stride;
  y += inst * stride;
  EGRID(idx, G.npts) y[idx] = x[idx] + m;
}

struct ELevel {
  int n = 0;
  int64_t npts = 0;
  double *xa = nullptr, *xb = nullptr, *r = nullptr, *b = nullptr;  // [count][npts]
};

struct EClass {
  int n = 0, count = 0, rpw = 4;
  int64_t npts = 0;
  std::vector<int> ids;  // instance indices (input order)
  int64_t base = 0;      // element offset of the class in the user's packed fields
  hipStream_t stream = nullptr;
  std::vector<ELevel> lv;
  double *r = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr, *work_b = nullptr,
         *work_p = nullptr;
  double *scal = nullptr, *partials = nullptr, *h_scal = nullptr;
  int* active = nullptr;        // device mask
  int* sel = nullptr;           // device selection for the final x updates
  // device-side convergence of a CG pass (ke_converge): per instance ||b||_W,
  // iteration count, buffer of the last p, relative recursive residual; two
  // flag pairs (active count, non-finite) read back alternately, pinned
  double* d_bn = nullptr;
  int* d_iters = nullptr;
  int* d_parity = nullptr;
  double* d_rel = nullptr;
  int* d_flags = nullptr;
  int* h_flags = nullptr;
  hipEvent_t ev_flags[2] = {nullptr, nullptr};
  std::vector<int> h_active;
  int32_t* clamped = nullptr;   // [count]
  EParam* prm = nullptr;        // [count]
  std::vector<EParam> h_prm;
  double* coef[2] = {nullptr, nullptr};     // [levels][count][kCoefStride] per operator
  TailArgs* tail[2] = {nullptr, nullptr};   // [count] per operator
  double* coarse[2] = {nullptr, nullptr};   // [count][400] per operator
  int degree[2] = {0, 0};
  std::vector<double> cvals;  // c of the CH operator per instance (for which tables were built)
  std::vector<double> h_coef0[2];           // level-0 records (host copy)
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  const double* graph_b[2] = {nullptr, nullptr};
  double* graph_z[2] = {nullptr, nullptr};
  int graph_rz[2] = {0, 0};
};

}  // namespace

struct bf_ensemble {
  int count = 0;
  hipStream_t stream = nullptr;
  std::vector<int32_t> sizes;
  std::vector<int64_t> offsets;  // per instance (input order)
  int64_t total = 0;
  std::vector<EClass> cls;
  std::vector<void*> allocs;
  std::vector<void*> host_allocs;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev2 = nullptr;  // end of a step on the caller's stream (timed from ev0)
};

namespace {

int efail(int code, const std::string& msg) { return host_fail(code, msg.c_str()); }

#define ECHK(expr)                                                                       \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return efail(BF_EHIP, std::string(#expr) + " failed: " + hipGetErrorString(e_));  \
  } while (0)
#define ETRY(expr)          \
  do {                      \
    int s_ = (expr);        \
    if (s_ < 0) return s_;  \
  } while (0)

template <typename T>
int ealloc(bf_ensemble* e, T** p, int64_t count) {
  void* ptr = nullptr;
  if (hipMalloc(&ptr, (size_t)(count > 0 ? count : 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return efail(BF_ENOMEM, "ensemble allocation failed");
  }
  e->allocs.push_back(ptr);
  *p = (T*)ptr;
  return BF_OK;
}

constexpr int kEnsPartials = 2 * 16384 + 4096;  // per class: reductions of all instances

// Sets the calling thread's batch context for a class (level l, operator op).
struct BatchScope {
  BatchScope(const EClass& C, int64_t stride, int64_t stride_c, const double* coef,
             const int* active, int rpw) {
    BatchCtx b;
    b.count = C.count;
    b.stride = stride;
    b.stride_c = stride_c;
    b.coef = coef;
    b.active = active;
    b.rpw = rpw;
    g_batch = b;
  }
  ~BatchScope() { g_batch = BatchCtx(); }
};

void set_sweep(int ia, int ig, int ia0) {
  g_batch.ia = ia;
  g_batch.ig = ig;
  g_batch.ia0 = ia0;
}

// Coefficient records of every level for operator op (c per instance); the
// device tables are allocated at creation.
int build_tables(EClass& C, int op, const std::vector<double>& c) {
  bf_solver_opts o;
  host_default_opts(op, &o);
  const int L = (int)C.lv.size();
  std::vector<double> tab((size_t)L * C.count * kCoefStride, 0.0);
  std::vector<TailArgs> tails(C.count);
  std::vector<double> coarse((size_t)C.count * kCoarseSize * kCoarseSize);
  int degree = 0;
  for (int k = 0; k < C.count; ++k) {
    for (int l = 0; l < L; ++l) {
      const int n = C.lv[l].n;
      double* rc = &tab[((size_t)l * C.count + k) * kCoefStride];
      const OpDesc A = host_level_op(op, n, c[k]);
      rc[0] = A.coef;
      rc[1] = A.dinv_int;
      rc[2] = A.dinv_edge;
      degree = host_smoother(op, n, c[k], o, rc + 3, rc + 11);
    }
    std::vector<double> G;
    ETRY(host_coarse_operator(op, c[k], G));
    std::copy(G.begin(), G.end(), coarse.begin() + (size_t)k * G.size());
  }
  // tail arguments: the levels n = 64, 32, 16, 8 of each instance (the tail
  // works on them in LDS; they are not part of the table above)
  for (int k = 0; k < C.count; ++k) {
    TailArgs& T = tails[k];
    T.nlev = 0;
    for (int n = std::min(C.n, kTailTop); n > kCoarseN; n /= 2) {
      const OpDesc A = host_level_op(op, n, c[k]);
      TailLevel& TL = T.lev[T.nlev++];
      TL.n = n;
      TL.coef = A.coef;
      TL.dinv_int = A.dinv_int;
      TL.dinv_edge = A.dinv_edge;
      TL.degree = host_smoother(op, n, c[k], o, TL.a, TL.g);
    }
    T.G = C.coarse[op] + (size_t)k * kCoarseSize * kCoarseSize;
  }
  ECHK(hipMemcpyAsync(C.coef[op], tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice,
                      C.stream));
  ECHK(hipMemcpyAsync(C.tail[op], tails.data(), tails.size() * sizeof(TailArgs),
                      hipMemcpyHostToDevice, C.stream));
  ECHK(hipMemcpyAsync(C.coarse[op], coarse.data(), coarse.size() * sizeof(double),
                      hipMemcpyHostToDevice, C.stream));
  ECHK(hipStreamSynchronize(C.stream));
  C.degree[op] = degree;
  C.h_coef0[op].assign(tab.begin(), tab.begin() + (size_t)C.count * kCoefStride);
  if (op == BF_OP_CH) C.cvals = c;
  if (C.graph[op]) {
    (void)hipGraphExecDestroy(C.graph[op]);
    C.graph[op] = nullptr;
  }
  return BF_OK;
}

const double* level_coef(const EClass& C, int op, int l) {
  return C.coef[op] + (size_t)l * C.count * kCoefStride;
}

// One V-cycle of every instance of the class on level l (b: level-l right
// hand sides, stride = the level's field size).  Returns the result buffer;
// rz_parts (level 0): partials of <b, z>_W written by the last sweep.
double* e_vcycle(EClass& C, int op, int l, const double* b, int* rz_parts) {
  ELevel& Lv = C.lv[l];
  hipStream_t st = C.stream;
  if (rz_parts) *rz_parts = 0;
  if (Lv.n <= kTailTop) {
    launch_tail_batch(op, C.tail[op], C.count, b, Lv.xa, Lv.npts, Lv.npts, st);
    return Lv.xa;
  }
  const int deg = C.degree[op];
  const int64_t sc = C.lv[l + 1].npts;
  BatchScope scope(C, Lv.npts, sc, level_coef(C, op, l), l == 0 ? C.active : nullptr, C.rpw);
  OpDesc A = host_level_op(op, Lv.n, 0.0);  // coefficients come from the batch records
  double* cur = Lv.xa;
  double* oth = Lv.xb;
  const bool streamed = stream_ok(Lv.n, 8);
  bool have_r = false;  // the residual of the pre-smoothed iterate is in Lv.r
  if (streamed && deg == 3 && smooth3_ok(Lv.n)) {
    // the three sweeps in one pass (weights from the instance records)
    set_sweep(0, 0, 0);
    stream_smooth3_from_zero<double>(A, b, cur, 0.0, 0.0, 0.0, 0.0, 0.0, st);
  } else if (streamed && deg == 2 && smooth3_ok(Lv.n)) {
    // both sweeps and the residual in one pass
    set_sweep(0, 0, 0);
    stream_smooth2_resid<double>(A, b, cur, Lv.r, 0.0, 0.0, 0.0, st);
    have_r = true;
  } else if (streamed && deg >= 2) {
    set_sweep(1, 1, 0);
    stream_smooth_from_zero<double>(A, b, cur, 0.0, 0.0, 0.0, st);
    for (int k = 2; k < deg; ++k) {
      set_sweep(k, k, 0);
      if (k == 2)
        stream_smooth_prev_from_b<double>(A, cur, b, oth, 0.0, 0.0, 0.0, st);
      else
        launch_smooth<double>(A, cur, oth, b, oth, 0.0, 0.0, st);
      std::swap(cur, oth);
    }
  } else {
    set_sweep(0, 0, 0);
    launch_smooth0<double>(A, b, cur, 0.0, st);
    for (int k = 1; k < deg; ++k) {
      set_sweep(k, k, 0);
      launch_smooth<double>(A, cur, k == 1 ? nullptr : oth, b, oth, 0.0, 0.0, st);
      std::swap(cur, oth);
    }
  }
  if (!have_r) launch_residual<double>(A, cur, b, Lv.r, nullptr, 0, st);
  launch_restrict<double>(Lv.n, Lv.r, C.lv[l + 1].b, st);
  double* ec = e_vcycle(C, op, l + 1, C.lv[l + 1].b, nullptr);
  // e_vcycle's scope ended: restore this level's batch context
  BatchScope scope2(C, Lv.npts, sc, level_coef(C, op, l), l == 0 ? C.active : nullptr, C.rpw);
  launch_prolong_add<double>(Lv.n, ec, cur, st);
  // the last two sweeps in one pass, into Lv.r (see vcycle_level)
  const bool pair = streamed && deg >= 2 && smooth_last2_ok(Lv.n);
  for (int k = 0; k < deg; ++k) {
    set_sweep(k, k, 0);
    if (pair && k == deg - 2) {
      if (rz_parts)
        *rz_parts = stream_smooth_last2_dot(A, cur, oth, b, Lv.r, 0.0, 0.0, 0.0, 0.0, C.partials,
                                            st) /
                    C.count;
      else
        stream_smooth_last2<double>(A, cur, oth, b, Lv.r, 0.0, 0.0, 0.0, 0.0, st);
      return Lv.r;
    }
    const double* prev = k == 0 ? nullptr : oth;
    if (rz_parts && k == deg - 1 && streamed)
      *rz_parts = stream_smooth_dot(A, cur, prev, b, oth, 0.0, 0.0, C.partials, st) / C.count;
    else
      launch_smooth<double>(A, cur, prev, b, oth, 0.0, 0.0, st);
    std::swap(cur, oth);
  }
  return cur;
}

// The level-0 V-cycle of the class, replayed from a captured graph.
double* e_precondition(EClass& C, int op, const double* r, int* rz_parts) {
  if (C.graph[op] && C.graph_b[op] == r) {
    if (hipGraphLaunch(C.graph[op], C.stream) == hipSuccess) {
      *rz_parts = C.graph_rz[op];
      return C.graph_z[op];
    }
  }
  if (C.graph[op]) {
    (void)hipGraphExecDestroy(C.graph[op]);
    C.graph[op] = nullptr;
  }
  hipStream_t user = C.stream, cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess &&
      hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    C.stream = cap;
    int rz = 0;
    double* z = e_vcycle(C, op, 0, r, &rz);
    C.stream = user;
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(cap, &graph) == hipSuccess && graph &&
        hipGraphInstantiate(&C.graph[op], graph, nullptr, nullptr, 0) == hipSuccess) {
      (void)hipGraphDestroy(graph);
      (void)hipStreamDestroy(cap);
      C.graph_b[op] = r;
      C.graph_z[op] = z;
      C.graph_rz[op] = rz;
      if (hipGraphLaunch(C.graph[op], C.stream) == hipSuccess) {
        *rz_parts = rz;
        return z;
      }
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    C.graph[op] = nullptr;
  } else if (cap) {
    (void)hipStreamDestroy(cap);
  }
  (void)hipGetLastError();
  C.stream = user;
  return e_vcycle(C, op, 0, r, rz_parts);
}

int e_read(EClass& C) {
  ECHK(hipMemcpyAsync(C.h_scal, C.scal, sizeof(double) * kNumSlots * C.count,
                      hipMemcpyDeviceToHost, C.stream));
  ECHK(hipStreamSynchronize(C.stream));
  return BF_OK;
}

void e_finalize(EClass& C, int64_t base, int np, int mode, int slot, const int* active) {
  hipLaunchKernelGGL(ke_finalize, dim3(C.count), dim3(kBlock), 0, C.stream, C.partials, base, np,
                     C.scal, mode, slot, (double)C.n * (double)C.n, active);
}

int e_dot_blocks(const EClass& C) {
  const int nb = red_blocks(C.npts);
  const int cap = 16384 / C.count;
  return std::max(1, std::min(nb, cap));
}

// W-dot of every instance into scal[slot] (diff: sum_W (x - y); mode F_MEAN: mean).
void e_wdot(EClass& C, const double* x, const double* y, int diff, int mode, int slot) {
  const Geo G = make_geo(C.n);
  const int nb = e_dot_blocks(C);
  hipLaunchKernelGGL(ke_dot, dim3(nb, C.count), dim3(kBlock), 0, C.stream, G, C.npts, x, y, diff,
                     C.partials);
  e_finalize(C, 0, nb, mode, slot, nullptr);
}

// One CG pass on the active instances of the class, from the current x and
// r = b - A x (r in C.r); a fresh Krylov space for all of them.  Leaves every
// instance's x complete (the deferred update applied) and its recursive
// residual and iteration count in stats.  Convergence is decided on the
// device after each r update (ke_converge): converged instances leave the
// mask that every kernel of the class honours, and the host reads only the
// count still active, after it has queued the next preconditioner
// application, so the class's stream never waits for the host.
int e_cg_pass(EClass& C, int op, const double* bn, double* x, const bf_solver_opts& o,
              std::vector<bf_solve_stats>& stats, std::vector<int>& ran) {
  hipStream_t st = C.stream;
  const Geo G = make_geo(C.n);
  const int B = C.count;
  ran.assign(B, 0);
  int remaining = 0;
  for (int k = 0; k < B; ++k) {
    ran[k] = C.h_active[k];
    remaining += C.h_active[k];
  }
  if (remaining == 0) return BF_OK;
  ECHK(hipMemcpyAsync(C.active, C.h_active.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
  ECHK(hipMemcpyAsync(C.d_bn, bn, sizeof(double) * B, hipMemcpyHostToDevice, st));
  launch_fill_i32(B, C.d_iters, 0, st);
  int rzp = 0;
  double* z = e_precondition(C, op, C.r, &rzp);
  e_finalize(C, 0, rzp, F_STORE, S_RZ, C.active);
  double* pcur = C.p;
  double* pnext = C.p2;
  bool first = true;
  int it = 0;
  const OpDesc A0 = host_level_op(op, C.n, 0.0);
  while (it < o.maxit) {
    {
      BatchScope scope(C, C.npts, 0, level_coef(C, op, 0), C.active, C.rpw);
      const int np = stream_cg_p(A0, z, pcur, pnext, C.q, x, C.scal, first, C.partials, st) / B;
      e_finalize(C, 0, np, F_ALPHA, 0, C.active);
    }
    std::swap(pcur, pnext);
    first = false;
    const int nb = e_dot_blocks(C);
    hipLaunchKernelGGL(ke_r_update, dim3(nb, B), dim3(kBlock), 0, st, G, C.npts, C.r, C.q, C.scal,
                       C.active, C.partials);
    e_finalize(C, 0, nb, F_STORE, S_RR, C.active);
    ++it;
    const int slot = it & 1;
    hipLaunchKernelGGL(ke_converge, dim3(1), dim3(kBlock), 0, st, C.scal, C.d_bn, o.rtol,
                       C.active, C.d_iters, C.d_parity, pcur == C.p ? 0 : 1, C.d_rel,
                       C.d_flags + 2 * slot, B);
    ECHK(hipMemcpyAsync(C.h_flags + 2 * slot, C.d_flags + 2 * slot, sizeof(int) * 2,
                        hipMemcpyDeviceToHost, st));
    ECHK(hipEventRecord(C.ev_flags[slot], st));
    if (it < o.maxit) {
      // the next application for the instances still active (the others are
      // masked); the count arrives while it runs
      z = e_precondition(C, op, C.r, &rzp);
      e_finalize(C, 0, rzp, F_BETA, 0, C.active);
    }
    ECHK(hipEventSynchronize(C.ev_flags[slot]));
    if (C.h_flags[2 * slot + 1]) return efail(BF_ENONFINITE, "residual norm is not finite");
    if (C.h_flags[2 * slot] == 0) break;
  }
  // per instance: iterations, recursive residual, the buffer of its last p
  // (instances stopped by maxit hold theirs in pcur)
  std::vector<int> iters(B), parity(B), act(B);
  std::vector<double> rel(B);
  ECHK(hipMemcpyAsync(iters.data(), C.d_iters, sizeof(int) * B, hipMemcpyDeviceToHost, st));
  ECHK(hipMemcpyAsync(parity.data(), C.d_parity, sizeof(int) * B, hipMemcpyDeviceToHost, st));
  ECHK(hipMemcpyAsync(act.data(), C.active, sizeof(int) * B, hipMemcpyDeviceToHost, st));
  ECHK(hipMemcpyAsync(rel.data(), C.d_rel, sizeof(double) * B, hipMemcpyDeviceToHost, st));
  ECHK(hipStreamSynchronize(st));
  for (int k = 0; k < B; ++k) {
    C.h_active[k] = 0;
    if (!ran[k]) continue;
    stats[k].iters += iters[k];
    stats[k].rel_res = rel[k];
    if (act[k]) parity[k] = (pcur == C.p) ? 0 : 1;
  }
  // the pending x += alpha p of every instance of the pass, from the buffer
  // that holds its last p
  for (int par = 0; par < 2; ++par) {
    std::vector<int> sel(B);
    for (int k = 0; k < B; ++k) sel[k] = (ran[k] && parity[k] == par) ? 1 : 0;
    ECHK(hipMemcpyAsync(C.sel + par * B, sel.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(ke_x_update, dim3(ew_blocks(C.npts), B), dim3(kBlock), 0, st, G, C.npts, x,
                       par == 0 ? C.p : C.p2, C.scal, C.sel + par * B);
  }
  return BF_OK;
}

// MG-preconditioned CG on every instance of the class (x starts at zero),
// then per instance: the constant-mode correction (CH), the double-double
// true residual and the status; an instance whose true residual is above
// rtol and above the floor bound of its iterate (floor_accept) restarts from that residual while
// each restart at least halves it (at most o.max_restarts), as on the
// single grid.
// guess: x holds a field on entry and every instance starts from gamma x,
// gamma = <b, A x>_W / <A x, A x>_W (the least-squares multiple; zero when
// that is not positive); otherwise from zero.
int e_solve(EClass& C, int op, const std::vector<double>& c, const double* b, double* x,
            const bf_solver_opts& o, std::vector<bf_solve_stats>& stats, bool guess) {
  hipStream_t st = C.stream;
  const Geo G = make_geo(C.n);
  const int B = C.count;
  if (op == BF_OP_CH && C.cvals != c) ETRY(build_tables(C, op, c));
  const OpDesc A0 = host_level_op(op, C.n, 0.0);
  if (guess) {
    {
      BatchScope scope(C, C.npts, 0, level_coef(C, op, 0), nullptr, C.rpw);
      launch_apply(A0, x, C.q, st);
    }
    e_wdot(C, b, C.q, 0, F_STORE, S_GB);
    e_wdot(C, C.q, C.q, 0, F_STORE, S_GG);
  }
  e_wdot(C, b, b, 0, F_STORE, S_BN2);
  ETRY(e_read(C));
  std::vector<double> bn(B), last(B, HUGE_VAL);
  std::vector<int> todo(B, 0);
  for (int k = 0; k < B; ++k) {
    const double v = C.h_scal[(size_t)k * kNumSlots + S_BN2];
    if (!std::isfinite(v)) return efail(BF_ENONFINITE, "right-hand side is not finite");
    bn[k] = std::sqrt(v);
    stats[k] = bf_solve_stats();
    stats[k].status = BF_OK;
    todo[k] = bn[k] > 0 ? 1 : 0;
    if (guess) {
      double* sc = C.h_scal + (size_t)k * kNumSlots;
      const double bq = sc[S_GB], qq = sc[S_GG];
      sc[S_GAMMA] = bq > 0.0 && qq > 0.0 && std::isfinite(bq / qq) ? bq / qq : 0.0;
    }
  }
  if (guess) {
    // the host copy of the scalars is current (read above): send it back with gamma
    ECHK(hipMemcpyAsync(C.scal, C.h_scal, sizeof(double) * kNumSlots * B, hipMemcpyHostToDevice,
                        st));
    hipLaunchKernelGGL(ke_scale, dim3(ew_blocks(C.npts), B), dim3(kBlock), 0, st, G, C.npts, x,
                       C.scal);
    BatchScope scope(C, C.npts, 0, level_coef(C, op, 0), nullptr, C.rpw);
    launch_residual_dd(A0, x, b, C.r, C.partials, 0, st);
  } else {
    launch_fill(C.npts * B, x, 0.0, st);
    launch_copy(C.npts * B, b, C.r, st);
  }
  const std::vector<double>& h_coef = C.h_coef0[op];
  std::vector<int> ran;
  for (;;) {
    C.h_active = todo;
    ETRY(e_cg_pass(C, op, bn.data(), x, o, stats, ran));
    ECHK(hipMemcpyAsync(C.sel, ran.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
    if (op == BF_OP_CH) {
      e_wdot(C, b, x, 1, F_MEAN, 0);
      hipLaunchKernelGGL(ke_add_mean, dim3(ew_blocks(C.npts), B), dim3(kBlock), 0, st, G,
                         C.npts, x, x, C.scal, 1.0, C.sel);
    }
    {
      // r = b - A x (double-double) of every instance; the next pass starts from it
      BatchScope scope(C, C.npts, 0, level_coef(C, op, 0), nullptr, C.rpw);
      const int np = launch_residual_dd(A0, x, b, C.r, C.partials, 0, st) / B;
      e_finalize(C, 0, np, F_STORE, S_RTRUE, nullptr);
      e_finalize(C, (int64_t)np * B, np, F_STORE, S_ULP2, nullptr);
    }
    ETRY(e_read(C));
    bool again = false;
    for (int k = 0; k < B; ++k) {
      if (!ran[k]) continue;
      bf_solve_stats& S = stats[k];
      OpDesc A = A0;
      A.coef = h_coef[(size_t)k * kCoefStride];
      const double* sc = C.h_scal + (size_t)k * kNumSlots;
      S.rel_res_true = std::sqrt(sc[S_RTRUE]) / bn[k];
      S.floor_est = std::sqrt(sc[S_ULP2] / 12.0 * host_column_sq(A)) / bn[k];
      if (!std::isfinite(S.rel_res_true)) return efail(BF_ENONFINITE, "true residual is not finite");
      todo[k] = 0;
      const bool hit_maxit = S.rel_res > o.rtol;
      // rounded additions to the iterate: one per CG iteration, plus the
      // constant-mode correction of each pass (see floor_accept)
      const double fb = floor_accept(S.floor_est, S.iters + S.restarts + 1);
      if (S.rel_res_true <= o.rtol) {
        S.status = BF_OK;
      } else if (hit_maxit) {
        S.status = BF_NOT_CONVERGED;
      } else if (S.rel_res_true <= fb) {
        S.status = BF_AT_FLOOR;
      } else if (S.restarts < o.max_restarts && S.rel_res_true < 0.5 * last[k]) {
        S.restarts++;
        last[k] = S.rel_res_true;
        todo[k] = 1;
        again = true;
      } else {
        S.status = S.rel_res_true <= 2.0 * fb ? BF_AT_FLOOR : BF_NOT_CONVERGED;
      }
    }
    if (!again) break;
  }
  return BF_OK;
}

}  // namespace

namespace {

// Solve, right-hand sides and projection of one class (all its instances).
int e_step_class(bf_ensemble* e, EClass& C, const bf_params* prm, double* phi,
                 const double* ustar, const double* vstar, double* p, double* u, double* v,
                 const bf_solver_opts& och, const bf_solver_opts& opr, bf_solve_stats* stats) {
  (void)e;
  hipStream_t st = C.stream;
  const int B = C.count;
  const Geo G = make_geo(C.n);
  const int64_t o = C.base;
  std::vector<EParam> hp(B);
  std::vector<double> c(B), zeros(B, 0.0);
  for (int k = 0; k < B; ++k) {
    const bf_params& P = prm[C.ids[k]];
    hp[k].dtMn2 = P.dt * P.M * (double)C.n * (double)C.n;
    hp[k].inv_npoly = 1.0 / P.Npoly;
    hp[k].chi = P.chi;
    hp[k].lo = P.phi_lo;
    hp[k].hi = P.phi_hi;
    hp[k].div_scale = (double)C.n / (2.0 * P.dt);
    hp[k].vel_scale = P.dt * (double)C.n * 0.5;
    c[k] = P.dt * P.M * P.kappa;
  }
  ECHK(hipMemcpyAsync(C.prm, hp.data(), sizeof(EParam) * B, hipMemcpyHostToDevice, st));
  launch_fill_i32(B, C.clamped, 0, st);
  // Cahn-Hilliard: b = phi + dt M L mu(phi), solve into phi from gamma phi
  static_assert(offsetof(EParam, dtMn2) == 0 && offsetof(EParam, hi) == 4 * sizeof(double),
                "the right-hand side reads dtMn2, inv_npoly, chi, lo, hi in this order");
  launch_ch_rhs_batch(C.n, B, C.npts, phi + o, C.work_b, reinterpret_cast<const double*>(C.prm),
                      (int)(sizeof(EParam) / sizeof(double)), C.clamped, st);
  std::vector<bf_solve_stats> sch(B), spr(B);
  ETRY(e_solve(C, BF_OP_CH, c, C.work_b, phi + o, och, sch, true));
  // pressure: rhs = div(u*)/dt, weighted mean removed; solve; mean of p removed
  hipLaunchKernelGGL(ke_divergence, dim3(ew_blocks(C.npts), B), dim3(kBlock), 0, st, G, C.npts,
                     C.prm, ustar + o, vstar + o, C.work_b);
  e_wdot(C, C.work_b, nullptr, 0, F_MEAN, 0);
  hipLaunchKernelGGL(ke_add_mean, dim3(ew_blocks(C.npts), B), dim3(kBlock), 0, st, G, C.npts,
                     C.work_b, C.work_p, C.scal, -1.0, nullptr);
  ETRY(e_solve(C, BF_OP_LAP, zeros, C.work_p, p + o, opr, spr, false));
  e_wdot(C, p + o, nullptr, 0, F_MEAN, 0);
  hipLaunchKernelGGL(ke_add_mean, dim3(ew_blocks(C.npts), B), dim3(kBlock), 0, st, G, C.npts,
                     p + o, p + o, C.scal, -1.0, nullptr);
  if (u && v)
    hipLaunchKernelGGL(ke_velocity, dim3(ew_blocks(C.npts), B), dim3(kBlock), 0, st, G, C.npts,
                       C.prm, p + o, ustar + o, vstar + o, u + o, v + o);
  std::vector<int32_t> cl(B);
  ECHK(hipMemcpyAsync(cl.data(), C.clamped, sizeof(int32_t) * B, hipMemcpyDeviceToHost, st));
  ECHK(hipStreamSynchronize(st));
  for (int k = 0; k < B; ++k) {
    const int id = C.ids[k];
    stats[2 * id] = sch[k];
    stats[2 * id].clamped = cl[k];
    stats[2 * id + 1] = spr[k];
  }
  return BF_OK;
}

// Tile height per class: time the class's float64 smoothing sweep (all its
// instances in one launch) with 4-, 5- and 8-row tiles and keep the fastest.
int autotune(EClass& C) {
  if (!stream_ok(C.n, 8)) return BF_OK;
  hipEvent_t a = nullptr, b = nullptr;
  ECHK(hipEventCreate(&a));
  ECHK(hipEventCreate(&b));
  const OpDesc A = host_level_op(BF_OP_LAP, C.n, 0.0);
  ELevel& L = C.lv[0];
  launch_fill(L.npts * C.count, L.xa, 0.0, C.stream);
  launch_fill(L.npts * C.count, L.xb, 0.0, C.stream);
  launch_fill(L.npts * C.count, L.b, 0.0, C.stream);
  float best = 1e30f;
  for (int rpw : {4, 5, 8}) {
    BatchScope scope(C, L.npts, 0, level_coef(C, BF_OP_LAP, 0), nullptr, rpw);
    set_sweep(1, 1, 0);
    for (int w = 0; w < 2; ++w) stream_smooth<double>(A, L.xa, L.xb, L.b, L.r, 0, 0, C.stream);
    ECHK(hipEventRecord(a, C.stream));
    for (int w = 0; w < 8; ++w) stream_smooth<double>(A, L.xa, L.xb, L.b, L.r, 0, 0, C.stream);
    ECHK(hipEventRecord(b, C.stream));
    ECHK(hipEventSynchronize(b));
    float ms = 0;
    ECHK(hipEventElapsedTime(&ms, a, b));
    if (ms < best) {
      best = ms;
      C.rpw = rpw;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return BF_OK;
}

int e_create(bf_ensemble* e, const int32_t* n, int count) {
  e->count = count;
  e->sizes.assign(n, n + count);
  // classes by size, ascending; instances keep their input order within a class
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return n[x] < n[y]; });
  e->offsets.assign(count, 0);
  int64_t off = 0;
  for (int k = 0; k < count;) {
    EClass C;
    C.n = n[order[k]];
    C.npts = (int64_t)(C.n + 1) * C.n;
    C.base = off;
    while (k < count && n[order[k]] == C.n) {
      e->offsets[order[k]] = off;
      C.ids.push_back(order[k]);
      off += C.npts;
      ++k;
    }
    C.count = (int)C.ids.size();
    e->cls.push_back(C);
  }
  e->total = off;
  for (EClass& C : e->cls) {
    const int B = C.count;
    if (B > 16384) return efail(BF_EINVAL, "too many instances of one size");
    ECHK(hipStreamCreateWithFlags(&C.stream, hipStreamNonBlocking));
    for (int m = C.n; m >= 8; m /= 2) {
      ELevel L;
      L.n = m;
      L.npts = (int64_t)(m + 1) * m;
      ETRY(ealloc(e, &L.xa, L.npts * B));
      ETRY(ealloc(e, &L.xb, L.npts * B));
      ETRY(ealloc(e, &L.r, L.npts * B));
      ETRY(ealloc(e, &L.b, L.npts * B));
      C.lv.push_back(L);
      if (m <= kTailTop) break;  // the tail works in LDS below its top level
    }
    ETRY(ealloc(e, &C.r, C.npts * B));
    ETRY(ealloc(e, &C.p, C.npts * B));
    ETRY(ealloc(e, &C.p2, C.npts * B));
    ETRY(ealloc(e, &C.q, C.npts * B));
    ETRY(ealloc(e, &C.work_b, C.npts * B));
    ETRY(ealloc(e, &C.work_p, C.npts * B));
    ETRY(ealloc(e, &C.scal, (int64_t)kNumSlots * B));
    ETRY(ealloc(e, &C.partials, kEnsPartials));
    ETRY(ealloc(e, &C.active, B));
    ETRY(ealloc(e, &C.sel, 2 * B));
    ETRY(ealloc(e, &C.d_bn, B));
    ETRY(ealloc(e, &C.d_iters, B));
    ETRY(ealloc(e, &C.d_parity, B));
    ETRY(ealloc(e, &C.d_rel, B));
    ETRY(ealloc(e, &C.d_flags, 4));
    for (int k = 0; k < 2; ++k)
      ECHK(hipEventCreateWithFlags(&C.ev_flags[k], hipEventDisableTiming));
    ETRY(ealloc(e, &C.clamped, B));
    ETRY(ealloc(e, &C.prm, B));
    const int L = (int)C.lv.size();
    for (int op = 0; op < 2; ++op) {
      ETRY(ealloc(e, &C.coef[op], (int64_t)L * B * kCoefStride));
      ETRY(ealloc(e, &C.tail[op], B));
      ETRY(ealloc(e, &C.coarse[op], (int64_t)B * kCoarseSize * kCoarseSize));
    }
    void* hs = nullptr;
    if (hipHostMalloc(&hs, sizeof(double) * kNumSlots * B) != hipSuccess)
      return efail(BF_ENOMEM, "pinned host allocation failed");
    e->host_allocs.push_back(hs);
    C.h_scal = (double*)hs;
    void* hf = nullptr;
    if (hipHostMalloc(&hf, sizeof(int) * 4) != hipSuccess)
      return efail(BF_ENOMEM, "pinned host allocation failed");
    e->host_allocs.push_back(hf);
    C.h_flags = (int*)hf;
    C.h_active.assign(B, 0);
    launch_fill((int64_t)kNumSlots * B, C.scal, 0.0, C.stream);
    launch_fill(C.npts * B, C.q, 0.0, C.stream);
    ETRY(build_tables(C, BF_OP_LAP, std::vector<double>(B, 0.0)));
    ETRY(build_tables(C, BF_OP_CH, std::vector<double>(B, 1e-7)));
    ETRY(autotune(C));
    ECHK(hipStreamSynchronize(C.stream));
  }
  ECHK(hipEventCreate(&e->ev0));
  ECHK(hipEventCreateWithFlags(&e->ev1, hipEventDisableTiming));
  ECHK(hipEventCreate(&e->ev2));
  return BF_OK;
}

}  // namespace

extern "C" {

int bf_ensemble_create(const int32_t* n, int32_t count, void* stream, bf_ensemble** out) {
  if (!n || !out || count < 1) return efail(BF_EINVAL, "null argument or count < 1");
  *out = nullptr;
  for (int i = 0; i < count; ++i)
    if (n[i] < 128 || n[i] > 8192 || (n[i] & (n[i] - 1)))
      return efail(BF_EINVAL, "ensemble sizes must be powers of two in [128, 8192]");
  bf_ensemble* e = new bf_ensemble();
  e->stream = (hipStream_t)stream;
  const int s = e_create(e, n, count);
  if (s != BF_OK) {
    bf_ensemble_destroy(e);
    return s;
  }
  *out = e;
  return BF_OK;
}

int bf_ensemble_destroy(bf_ensemble* e) {
  if (!e) return BF_OK;
  for (EClass& C : e->cls) {
    if (C.stream) (void)hipStreamSynchronize(C.stream);
    for (int op = 0; op < 2; ++op)
      if (C.graph[op]) (void)hipGraphExecDestroy(C.graph[op]);
    for (int k = 0; k < 2; ++k)
      if (C.ev_flags[k]) (void)hipEventDestroy(C.ev_flags[k]);
    if (C.stream) (void)hipStreamDestroy(C.stream);
  }
  for (void* p : e->allocs) (void)hipFree(p);
  for (void* p : e->host_allocs) (void)hipHostFree(p);
  if (e->ev0) (void)hipEventDestroy(e->ev0);
  if (e->ev1) (void)hipEventDestroy(e->ev1);
  if (e->ev2) (void)hipEventDestroy(e->ev2);
  delete e;
  return BF_OK;
}

int bf_ensemble_layout(const bf_ensemble* e, int64_t* offsets, int64_t* total) {
  if (!e) return efail(BF_EINVAL, "null ensemble");
  if (offsets) std::copy(e->offsets.begin(), e->offsets.end(), offsets);
  if (total) *total = e->total;
  return BF_OK;
}

int bf_ensemble_info(const bf_ensemble* e, int32_t* nclasses, int32_t* class_n,
                     int32_t* class_count, int32_t* class_rpw) {
  if (!e) return efail(BF_EINVAL, "null ensemble");
  if (nclasses) *nclasses = (int32_t)e->cls.size();
  for (size_t k = 0; k < e->cls.size(); ++k) {
    if (class_n) class_n[k] = e->cls[k].n;
    if (class_count) class_count[k] = e->cls[k].count;
    if (class_rpw) class_rpw[k] = e->cls[k].rpw;
  }
  return BF_OK;
}

int bf_ensemble_step(bf_ensemble* e, const bf_params* prm, double* phi, const double* ustar,
                     const double* vstar, double* p, double* u, double* v,
                     const bf_solver_opts* ch, const bf_solver_opts* pr, bf_solve_stats* stats,
                     double* ms) {
  if (!e || !prm || !phi || !ustar || !vstar || !p || !stats)
    return efail(BF_EINVAL, "null argument");
  if ((u == nullptr) != (v == nullptr)) return efail(BF_EINVAL, "u and v must both be given or both be null");
  for (int i = 0; i < e->count; ++i) {
    const bf_params& P = prm[i];
    if (!(P.dt > 0) || !(P.Npoly > 0) || !(P.phi_lo > 0) || !(P.phi_hi < 1) ||
        !(P.phi_lo < P.phi_hi) || !(P.M >= 0) || !(P.kappa >= 0))
      return efail(BF_EINVAL, "bad parameters of instance " + std::to_string(i));
  }
  bf_solver_opts och, opr;
  host_default_opts(BF_OP_CH, &och);
  host_default_opts(BF_OP_LAP, &opr);
  if (ch) och = *ch;
  if (pr) opr = *pr;
  ETRY(host_check_opts(och));
  ETRY(host_check_opts(opr));
  if (och.ksp != BF_KSP_CG || och.pc != BF_PC_MG || opr.ksp != BF_KSP_CG || opr.pc != BF_PC_MG ||
      och.mg_precision != BF_MG_F64 || opr.mg_precision != BF_MG_F64 || och.degree || opr.degree ||
      och.ratio > 0 || opr.ratio > 0 || och.smoother != BF_SMOOTH_CHEBYSHEV ||
      opr.smoother != BF_SMOOTH_CHEBYSHEV)
    return efail(BF_EUNSUPPORTED,
                 "the ensemble runs float64 CG with the default multigrid (rtol, maxit only)");
  // every class waits for the caller's stream, the caller's stream for every class
  ECHK(hipEventRecord(e->ev0, e->stream));
  for (EClass& C : e->cls) ECHK(hipStreamWaitEvent(C.stream, e->ev0, 0));
  std::vector<int> rc(e->cls.size(), BF_OK);
  std::vector<std::string> err(e->cls.size());
  if (e->cls.size() == 1) {
    rc[0] = e_step_class(e, e->cls[0], prm, phi, ustar, vstar, p, u, v, och, opr, stats);
  } else {
    std::vector<std::thread> th;
    for (size_t k = 0; k < e->cls.size(); ++k)
      th.emplace_back([&, k] {
        rc[k] = e_step_class(e, e->cls[k], prm, phi, ustar, vstar, p, u, v, och, opr, stats);
        if (rc[k] < 0) err[k] = bf_last_error();
      });
    for (auto& t : th) t.join();
  }
  for (size_t k = 0; k < e->cls.size(); ++k)
    if (rc[k] < 0) return efail(rc[k], err[k].empty() ? "ensemble step failed" : err[k]);
  for (EClass& C : e->cls) {
    ECHK(hipEventRecord(e->ev1, C.stream));
    ECHK(hipStreamWaitEvent(e->stream, e->ev1, 0));
  }
  // device time of the step: from the marker every class waited for to the
  // marker that waited for every class, both on the caller's stream
  ECHK(hipEventRecord(e->ev2, e->stream));
  ECHK(hipStreamSynchronize(e->stream));
  if (ms) {
    float dev_ms = 0.0f;
    ECHK(hipEventElapsedTime(&dev_ms, e->ev0, e->ev2));
    *ms = dev_ms;
  }
  int worst = BF_OK;
  for (int i = 0; i < 2 * e->count; ++i) worst = std::max(worst, (int)stats[i].status);
  return worst;
}

}  // extern "C"
