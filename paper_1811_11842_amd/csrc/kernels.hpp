// Launchers of the device kernels (host-callable, asynchronous on `st`).
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace bf {

// Operator of one grid level: y = A x.
//   OP_LAP: A = L (5-point), coef = n^2
//   OP_CH : A = I + s * S13 with S13 the integer 13-point stencil, s = c n^4
struct OpDesc {
  int op;          // 0 = Laplacian, 1 = Cahn-Hilliard, 2 = Helmholtz with Dirichlet walls
  int n;
  double coef;     // n^2 (LAP), s = c n^4 (CH) or s = beta n^2 (Helmholtz)
  double dinv_int; // 1 / diag on ordinary rows
  double dinv_edge;// 1 / diag on rows 1 and n-1 (CH); 0 on the wall rows (Helmholtz)
};

// Batches of equal-sized instances (the ensemble driver).  While a thread's
// batch context has count > 1, the launchers below that support batches run
// every field operation on `count` instances stored `stride` elements apart
// (coarse fields of transfers: `stride_c`), with per-instance coefficient
// records (`coef`, kCoefStride doubles each: coef, dinv_int, dinv_edge,
// a[8], g[8]; a = a[ia], g = g[ig], a0 = a[ia0] for smoothing sweeps) and
// per-instance device scalars kNumSlots apart; reductions return the
// partial count of all instances (instance i owns the i-th equal share).
constexpr int kCoefStride = 20;
// Relative true residual at which a Krylov iterate counts as at its float64
// floor: floor_est is the residual of one rounding of every entry (uniform,
// variance ulp^2/12); an iterate built by `updates` rounded additions (CG: one
// per iteration, plus the constant-mode correction) carries about sqrt(updates)
// such roundings (a random walk: measured 3.75 floor_est after 14 CG updates
// at 4096^2, against sqrt(15) = 3.87), so the bound is 1.5 sqrt(updates + 1)
// floor_est, with updates capped at 64 (long runs are not given a looser bound
// than about 12 floor_est).  The recursive residual has then met rtol, and
// what is left is that rounding noise, which A^{-1} damps: no refinement
// restart is needed.
inline double floor_accept(double floor_est, int updates) {
  const int k = updates < 0 ? 0 : (updates > 64 ? 64 : updates);
  return 1.5 * std::sqrt((double)k + 1.0) * floor_est;
}

struct BatchCtx {
  int count = 1;
  int64_t stride = 0, stride_c = 0;
  const double* coef = nullptr;
  int ia = 0, ig = 0, ia0 = 0;
  const int* active = nullptr;
  int rpw = 0;  // stencil tile height for this batch (0: default)
};
extern thread_local BatchCtx g_batch;

// Launch shape of the tiled stencil kernels (stream.hip), two values per
// lane, 128 columns per wavefront; used for grid levels with n >= 128,
// smaller levels use the one-thread-per-node kernels.
constexpr int kStreamMaxBlocks = 16384;  // workgroups per launch; beyond, wavefronts loop over tiles
struct StreamCfg {
  int rpw;      // output rows per wavefront tile
  int wstrips;  // column strips of 128 columns
  int rgroups;  // row groups of rpw rows
  int tiles;    // wstrips * rgroups (one wavefront each)
  int blocks;   // workgroups of 4 wavefronts (capped; wavefronts then loop)
};
bool stream_ok(int n);              // float64 fields
StreamCfg stream_cfg(int n);
bool stream_ok(int n, int elem_bytes);
StreamCfg stream_cfg(int n, int elem_bytes);
StreamCfg stream_cfg(int n, int elem_bytes, bool apply);  // apply: y = A x kernels
int stream_apply(const OpDesc& A, const double* x, double* y, hipStream_t st);
int stream_apply_dot(const OpDesc& A, const double* p, double* q, double* partials, bool dd,
                     hipStream_t st);
template <typename T>
int stream_residual(const OpDesc& A, const T* x, const T* b, T* r, double* partials,
                    hipStream_t st);
// r32 (optional): also receives (float) r (the float32 V-cycle's input).
int stream_residual_dd(const OpDesc& A, const double* x, const double* b, double* r,
                       double* partials, hipStream_t st, float* r32 = nullptr);
// Partials of <b, A x>_W, <A x, A x>_W and <b, b>_W (three groups of the
// returned count, in that order) without writing A x: the least-squares
// initial guess and ||b||_W in one pass.
int stream_guess(const OpDesc& A, const double* x, const double* b, double* partials,
                 hipStream_t st);
template <typename T>
void stream_smooth(const OpDesc& A, const T* x, const T* xprev, const T* b, T* xout, double a,
                   double g, hipStream_t st);
// Two sweeps from a zero guess in one pass: x1 = a0 D^{-1} b is formed on
// load, xout = x1 + a1 D^{-1}(b - A x1) + g1 x1.
template <typename T>
void stream_smooth_from_zero(const OpDesc& A, const T* b, T* xout, double a0, double a1,
                             double g1, hipStream_t st);
// xout = x + a D^{-1}(b - A x) + g (x - x1), x1 = a0 D^{-1} b formed on the fly.
template <typename T>
void stream_smooth_prev_from_b(const OpDesc& A, const T* x, const T* b, T* xout, double a0,
                               double a, double g, hipStream_t st);
// Three sweeps from a zero guess in one pass (single grids, streamed levels):
// x1 = a0 D^{-1} b, x2 = x1 + a1 D^{-1}(b - A x1) + g1 x1,
// xout = x2 + a2 D^{-1}(b - A x2) + g2 (x2 - x1).
bool smooth3_ok(int n);
template <typename T>
void stream_smooth3_from_zero(const OpDesc& A, const T* b, T* xout, double a0, double a1,
                              double g1, double a2, double g2, hipStream_t st);
// Two sweeps from a zero guess and the residual, in one pass (degree-2
// smoothers): x1 = a0 D^{-1} b, xout = x1 + a1 D^{-1}(b - A x1) + g1 x1,
// r = b - A xout.
template <typename T>
void stream_smooth2_resid(const OpDesc& A, const T* b, T* xout, T* r, double a0, double a1,
                          double g1, hipStream_t st);
// The same three sweeps followed by r = b - A xout, in one pass (float32).
bool smooth3r_ok(int n, int elem_bytes);
template <typename T>
void stream_smooth3_resid(const OpDesc& A, const T* b, T* xout, T* r, double a0, double a1,
                          double g1, double a2, double g2, hipStream_t st);
// The last two sweeps of a smoother in one pass (single grids, streamed
// levels): x2 = x1 + a1 D^{-1}(b - A x1) + g1 (x1 - x0),
// xout = x2 + a2 D^{-1}(b - A x2) + g2 (x2 - x1); xout aliases neither x1
// nor x0 (x0 unused when g1 == 0).  The _dot forms also leave partials of
// <b, xout>_W (and of <xout, q>_W) and return their count.
bool smooth_last2_ok(int n);
template <typename T>
void stream_smooth_last2(const OpDesc& A, const T* x1, const T* x0, const T* b, T* xout,
                         double a1, double g1, double a2, double g2, hipStream_t st);
int stream_smooth_last2_dot(const OpDesc& A, const double* x1, const double* x0, const double* b,
                            double* xout, double a1, double g1, double a2, double g2,
                            double* partials, hipStream_t st);
int stream_smooth_last2_dot2(const OpDesc& A, const float* x1, const float* x0, const float* b,
                             double* xout, const double* q, double a1, double g1, double a2,
                             double g2, double* partials, hipStream_t st);
int stream_smooth_last2_dot2_f32(const OpDesc& A, const float* x1, const float* x0,
                                 const float* b, float* xout, const double* q, double a1,
                                 double g1, double a2, double g2, double* partials,
                                 hipStream_t st);
// Float32 smoothing sweep writing a float64 result, with partials of <b, out>_W
// (partials[0..np)) and <out, q>_W (partials[np..2 np)); returns np.
int stream_smooth_dot2(const OpDesc& A, const float* x, const float* xprev, const float* b,
                       double* xout, const double* q, double a, double g, double* partials,
                       hipStream_t st);
// The same sweep writing z in float32 (the CG step then reads it with
// stream_cg_p32; z is a float32 result, so nothing is lost).
int stream_smooth_dot2_f32(const OpDesc& A, const float* x, const float* xprev, const float* b,
                           float* xout, const double* q, double a, double g, double* partials,
                           hipStream_t st);
// The CG step reading the float32 z: the search direction p' = z + beta p_old
// is rounded to float32 and kept in float32 (p_old, p_new); q = A p', the
// reduction <p', q>_W and the deferred x += alpha p_old use the rounded p',
// so the iterate and the recursive residual stay consistent with each other.
// x null: the step leaves x alone (the caller applies x += alpha p in batches).
int stream_cg_p32(const OpDesc& A, const float* z, const float* p_old, float* p_new, double* q,
                  double* x, const double* scal, bool first, double* partials, hipStream_t st);
// Smoothing sweep that also writes partials of <b, xout>_W; returns their count.
int stream_smooth_dot(const OpDesc& A, const double* x, const double* xprev, const double* b,
                      double* xout, double a, double g, double* partials, hipStream_t st);
// One CG step on the operator: p_new = z + beta p_old (p_new = z if first),
// q = A p_new (double-double for the CH operator), partials of <p_new, q>_W,
// and the deferred x += alpha p_old (skipped if first); alpha, beta are read
// from scal[S_ALPHA], scal[S_BETA].  p_new must not alias p_old or z.  Returns
// the number of partials.
int stream_cg_p(const OpDesc& A, const double* z, const double* p_old, double* p_new, double* q,
                double* x, const double* scal, bool first, double* partials, hipStream_t st);
int launch_cg_p(const OpDesc& A, const double* z, const double* p_old, double* p_new, double* q,
                double* x, const double* scal, bool first, double* partials, int nparts,
                hipStream_t st);
// r -= alpha q (alpha = scal[S_ALPHA]), partials of ||r||_W^2; if r32 is
// given, also r32 = (float) r.
void launch_r_update(int n, double* r, const double* q, const double* scal, double* partials,
                     int nparts, hipStream_t st, float* r32 = nullptr);
// x += alpha p (alpha = scal[S_ALPHA]).
void launch_x_update(int n, double* x, const double* p, const double* scal, hipStream_t st);
void launch_x_update(int n, double* x, const float* p, const double* scal, hipStream_t st);
// x += sum_{i < m} alpha[i] p[i] (m <= kRing float32 fields, alpha on the device).
void launch_x_accum(int n, double* x, const float* const* p, int m, const double* alpha,
                    hipStream_t st);
// The coarse-grid correction and the whole post-smoother of a level in one
// pass: x0 = x + P e (e the coarse correction), then `degree` sweeps
// x_{k+1} = x_k + a[k] D^{-1}(b - A x_k) + g[k] (x_k - x_{k-1}) (g[0] unused);
// out = x_degree (must not alias x, e or b).  The _dot forms also leave
// partials of <b, out>_W (and of <out, q>_W) and return their count.
bool post_ok(int n, int op, int degree, double g0, int elem_bytes);
// The correction and the first post-sweep only (13-point operator, float64
// levels where post_ok is false): x1 = sweep(x0), x0 = x + P e; writes both.
bool post1_ok(int n, int op, int degree, double g0);
template <typename T>
void stream_post1(const OpDesc& A, const T* x, const T* e, const T* b, T* x1, T* x0, double a0,
                  hipStream_t st);
template <typename T>
void stream_post(const OpDesc& A, int degree, const T* x, const T* e, const T* b, T* out,
                 const double* a, const double* g, hipStream_t st);
int stream_post_dot(const OpDesc& A, int degree, const double* x, const double* e,
                    const double* b, double* out, const double* a, const double* g,
                    double* partials, hipStream_t st);
// q null: the partials of <b, z>_W only (q is not read)
int stream_post_dot2(const OpDesc& A, int degree, const float* x, const float* e, const float* b,
                     double* out, const double* q, const double* a, const double* g,
                     double* partials, hipStream_t st);
int stream_post_dot2_f32(const OpDesc& A, int degree, const float* x, const float* e,
                         const float* b, float* out, const double* q, const double* a,
                         const double* g, double* partials, hipStream_t st);
bool transfer_stream_ok(int nf);
template <typename T>
void stream_prolong_add(int nf, const T* coarse, T* fine, hipStream_t st);
template <typename T>
void stream_restrict(int nf, const T* fine, T* coarse, hipStream_t st);

// Coarse tail: all levels 8 <= n <= kTailTop plus the exact 5 x 4 solve in
// one workgroup with the fields in LDS (tail.hip): three fields per level
// (two iterates, right-hand side), 16720 elements = 134 KB in float64.
constexpr int kTailTop = 64;
constexpr int kTailMaxLevels = 4;      // n = 64, 32, 16, 8
constexpr int kTailMaxDoubles = 16720; // 3 (65*64 + 33*32 + 17*16 + 9*8) + 2 * 20
struct TailLevel {
  int n;
  int degree;
  double coef, dinv_int, dinv_edge;
  double a[8], g[8];
};
struct TailArgs {
  int nlev;                       // smoothing levels (top n down to 8)
  TailLevel lev[kTailMaxLevels];  // lev[0] is the top (finest) tail level
  const double* G;                // dense solve of the 5 x 4 grid (20 x 20, row-major)
};
template <typename T>
void launch_tail(int op, const TailArgs& P, const T* b_in, T* x_out, hipStream_t st);
// Batched tail: args (device, count entries) per instance; fields sin / sout apart.
template <typename T>
void launch_tail_batch(int op, const TailArgs* args, int count, const T* b_in, T* x_out,
                       int64_t sin, int64_t sout, hipStream_t st);

// The launchers that write reduction partials return how many they wrote
// (the count the matching launch_finalize must reduce); `nparts` is the
// count used by the one-thread-per-node fallback.
void launch_apply(const OpDesc& A, const double* x, double* y, hipStream_t st);
// q = A p and per-block partials of <p, q>_W; accurate = double-double stencil sum.
int launch_apply_dot(const OpDesc& A, const double* p, double* q, double* partials,
                     int nparts, hipStream_t st, bool accurate);
// r = b - A x (x == nullptr means x = 0); partials of ||r||_W^2 if partials != nullptr.
template <typename T>
int launch_residual(const OpDesc& A, const T* x, const T* b, T* r, double* partials, int nparts,
                    hipStream_t st);
// r = b - A x evaluated with a double-double stencil sum (accurate to a few
// ulps of r); partials[0..np) of ||r||_W^2 and partials[np..2 np) of
// sum_W ulp(x)^2, np = the returned count.
int launch_residual_dd(const OpDesc& A, const double* x, const double* b, double* r,
                       double* partials, int nparts, hipStream_t st);
// xout = x + a D^{-1}(b - A x) + g (x - xprev); xprev == nullptr means 0.
// xout may alias xprev, not x.
template <typename T>
void launch_smooth(const OpDesc& A, const T* x, const T* xprev, const T* b, T* xout, double a,
                   double g, hipStream_t st);
// xout = a D^{-1} b (first sweep from a zero guess).
template <typename T>
void launch_smooth0(const OpDesc& A, const T* b, T* xout, double a, hipStream_t st);
// z = D^{-1} r (Jacobi preconditioner).
void launch_jacobi_pc(const OpDesc& A, const double* r, double* z, hipStream_t st);

template <typename T>
void launch_restrict(int nf, const T* fine, T* coarse, hipStream_t st);
template <typename T>
void launch_prolong_add(int nf, const T* coarse, T* fine, hipStream_t st);
// x = G b on the coarsest grid (dense size x size matrix, row-major, float64).
template <typename T>
void launch_coarse_solve(int size, const double* G, const T* b, T* x, hipStream_t st);
// y = (float) x
void launch_to_float(int64_t count, const double* x, float* y, hipStream_t st);
// y = (double) x
void launch_to_double(int64_t count, const float* x, double* y, hipStream_t st);

// partials of <x, y>_W (y == nullptr means y = 1: weighted sum of x).
void launch_dot(int n, const double* x, const double* y, double* partials, int nparts,
                hipStream_t st);
// partials of sum_W (x - y)
void launch_wsum_diff(int n, const double* x, const double* y, double* partials, int nparts,
                      hipStream_t st);
// Reduce partials in a fixed order and update scalars (see FinalizeMode);
// host (F_STORE only): pinned host scalars that also receive scal[slot] and,
// after it, hseq in host[S_HSEQ].
void launch_finalize(const double* partials, int nparts, double* scal, int mode, int slot,
                     int n, hipStream_t st, double* host = nullptr, double hseq = 0.0);
// Norms of a residual from the scalars of its reductions (scal[S_BN2] =
// ||b||_W^2, scal[S_RTRUE] = ||r||_W^2, scal[S_ULP2] = sum_W ulp(x)^2):
// out[0] = ||r||_W / ||b||_W, out[1] = sqrt(scal[S_ULP2] / 12 * csq) / ||b||_W
// (the float64 floor estimate), out[2] = ||b||_W; ||b||_W = 0 divides by 1.
void launch_residual_norms(const double* scal, double csq, double* out, hipStream_t st);
// Flexible CG: scal[S_RZ] = rho (partials[0..np)), scal[S_BETA] =
// -scal[S_ALPHA] * gamma / rho_old with gamma = sum partials[np..2 np).
void launch_finalize_flex(const double* partials, int nparts, double* scal, hipStream_t st);
// y = x - scal[S_MEAN]
void launch_sub_mean(int n, const double* x, double* y, const double* scal, hipStream_t st);
// b = r = x - scal[S_MEAN], r32 = (float) b when given, nparts partials of
// ||b||_W^2: the start of a solve from x = 0 with a projected right-hand side.
void launch_project_start(int n, const double* x, double* b, double* r, float* r32,
                          const double* scal, double* partials, int nparts, hipStream_t st);
// y = x + scal[S_MEAN]
void launch_add_mean(int n, const double* x, double* y, const double* scal, hipStream_t st);
void launch_fill(int64_t count, double* x, double v, hipStream_t st);
void launch_copy(int64_t count, const double* x, double* y, hipStream_t st);
void launch_fill_i32(int count, int32_t* x, int32_t v, hipStream_t st);
// y = x, 16-byte accesses (count even, pointers 16-byte aligned).
void launch_copy2(int64_t count, const double* x, double* y, hipStream_t st);

// Step pieces.
// Coefficients of the Flory-Huggins right-hand side: dtM n^2, 1/N, chi, clamp.
struct RhsCoef {
  double dtMn2, inv_npoly, chi, lo, hi;
};
// b = base + dtM L mu_FH(clamp(phi*)), phi* = phi (prev null) or 3/2 phi - 1/2 prev;
// mu_ws: a field of workspace (used below 128 columns only); base may alias b;
// clamped nodes counted into clamp_count.
void launch_ch_rhs(int n, const double* phi, const double* prev, const double* base, double* b,
                   double* mu_ws, double dtM, double inv_npoly, double chi, double lo, double hi,
                   int32_t* clamp_count, hipStream_t st);
// The same (prev null, base = phi) for `count` instances of n >= 128 stored
// `stride` apart: instance i reads its coefficients (dtM n^2, 1/N, chi, lo,
// hi) from icoef + i icoef_stride (device) and counts into clamp_counts[i].
void launch_ch_rhs_batch(int n, int count, int64_t stride, const double* phi, double* b,
                         const double* icoef, int icoef_stride, int32_t* clamp_counts,
                         hipStream_t st);
void launch_divergence(int n, const double* u, const double* v, double* rhs, double scale,
                       hipStream_t st);
// Variable-mobility Cahn-Hilliard operator A_m = I + c L_m L (double-double
// evaluation): y = A_m x (b == nullptr) or y = b - A_m x with partials of
// ||y||_W^2 and of sum_W ulp(x)^2 times the local squared column norm (two
// groups; returns the group size).
int launch_mob(int n, double c, const double* m, const double* x, const double* b, double* y,
               double* partials, int nparts, hipStream_t st);
// Variable-mobility V-cycle pieces (plain T arithmetic, one node per
// thread; cs = c n^4 of the level, m the level's node mobilities):
// Chebyshev/Jacobi sweep, first sweep from zero, residual, and injection of
// m onto the next coarser level.
template <typename T>
void launch_mob_smooth(int n, double cs, const T* m, const T* x, const T* xprev, const T* b,
                       T* xout, double a, double g, hipStream_t st);
template <typename T>
void launch_mob_smooth0(int n, double cs, const T* m, const T* b, T* xout, double a0,
                        hipStream_t st);
template <typename T>
void launch_mob_residual(int n, double cs, const T* m, const T* x, const T* b, T* r,
                         hipStream_t st);
template <typename T>
void launch_inject(int nf, const T* fine, T* coarse, hipStream_t st);
// m = M clamp(phi); mu_ws = mu_FH(clamp(phi)); b = phi + dt L_m mu_ws.
void launch_mob_rhs(int n, const double* phi, double* m, double* mu_ws, double* b, double M,
                    double dt, double inv_npoly, double chi, double lo, double hi,
                    int32_t* clamp_count, hipStream_t st);
void launch_momentum_rhs(int n, const double* u, const double* v, double dt, double e, double U,
                         double* bu, double* bv, hipStream_t st);
void launch_velocity(int n, const double* p, const double* us, const double* vs, double* u,
                     double* v, double scale, hipStream_t st);

// Advection and adjoint pieces.
// b -= dt D(phi; u, v), D = div_h(phi u, phi v), phi even and v odd across the walls.
void launch_advect_sub(int n, const double* phi, const double* u, const double* v, double* b,
                       double dt, hipStream_t st);
// y = x w_j (inverse false) or x / w_j (inverse true); trapezoid row weights.
void launch_wscale(int n, const double* x, double* y, bool inverse, hipStream_t st);
struct AdjCoef {
  double dt, dtM, inv_npoly, chi, lo, hi;
};
// lam = eta + dtM mu'(phi) L^T eta - dt D^T eta from e = W^{-1} eta (u, v may be
// null: no advection; du, dv may be null: no U term); partials[0..nparts) of
// sum L^T eta (1 - 2 clamp(phi)), partials[nparts..2 nparts) of sum eta D(phi; du, dv).
void launch_adjoint_rhs(int n, const double* e, const double* phi, const double* u,
                        const double* v, const double* du, const double* dv, double* lam,
                        const AdjCoef& C, double* partials, int nparts, hipStream_t st);

// GMRES pieces (weighted inner products).
// partials[k * nparts + b] of <V_k, w>_W for k < m (V: m vectors of npts each).
void launch_mdot(int n, const double* V, int m, const double* w, double* partials, int nparts,
                 hipStream_t st);
// Reduce m groups of partials: scal[slot + k] = sum_b partials[k * nparts + b].
void launch_finalize_multi(const double* partials, int nparts, int m, double* scal, int slot,
                           hipStream_t st);
// w -= sum_k h[k] V_k (h = scal + slot), and partials of ||w||_W^2.
void launch_maxpy(int n, const double* V, int m, const double* h, double* w, double* partials,
                  int nparts, hipStream_t st);
// x += sum_k y[k] Z_k with y = host-provided coefficients (device array).
void launch_axpy_multi(int n, const double* Z, int m, const double* y, double* x,
                       hipStream_t st);
// y = a * x
void launch_scale(int n, const double* x, double* y, const double* scal, int slot, int invert_sqrt,
                  hipStream_t st);

}  // namespace bf
