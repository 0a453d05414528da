// Device kernels of the exact real-time step: the bounded QP of eq. (qp_rto)
// in w = (u, s), solved by a primal-dual interior-point method with
// Mehrotra's predictor-corrector (Section IV-B.1/2: barrier subproblem
// eq. ipm_subproblem, Newton system eq. ipm_kkt_reduced).  The QP's data
// are the scaled AL derivatives (eq. gradient_auglag, eq. hessian_auglag,
// Section IV-A.2):
//   g = (grad_u, -D_c (y + rho D_c (c - s))),
//   Hw = [[H + delta I, -rho J^T D_c^2], [-rho D_c^2 J, rho D_c^2]],
// H the reduced Hessian, J = grad_u c the reduced Jacobian.  Every Newton
// system (Hw + Sigma) x = b is solved through the Schur complement of
// Proposition 3 (eq. ipm_kkt_schur, eq. schur_matrix) with
// C = rho sigma^2 + Sigma_s (diagonal):
//   x_u = S^{-1} (b_u + rho J^T (sigma^2 b_s / C)),
//   x_s = (b_s + rho sigma^2 (J x_u)) / C,
//   S = H + delta I + Sigma_u - rho^2 J^T diag(sigma^4 / C) J
//     = H_gn + delta I + Sigma_u,
// where H_gn is the reduced Hessian with each constraint's curvature weight
// rho sigma_k^2 replaced by rho sigma_k^2 Sigma_s,k / C_k (it is formed by
// the batched Hessian-vector products, not from J).
//
// Inertia control (Section IV-B.2: the regularisation keeps the Newton
// matrix, hence S, positive definite): the Cholesky runs on S + w I, first
// with w = 0 if the last successful w was 0, else max(w0, w_last /
// QP_REG_DOWN); a failed factorization raises w (w0, then QP_REG_UP times)
// and the next slot retries with the same S; w0 = QP_REG_BASE max(1, max
// |diag H|).  Every factorization attempt takes one of the host's slots.
//
// The iteration is predicated on the device: `done` is 0 while it runs,
// 1 once the KKT error is below tol, 2 when it is not finite, 16 + column
// when w passes QP_REG_MAX (column of the last failed Cholesky) and -1 when
// a triangular-solve workgroup gave up waiting; every kernel of a later
// step returns at once.  Within a slot, skF (done or retrying) skips the
// fresh part (KKT test, assembly of S) and sk2 (done or the factorization
// failed) the solves and steps.  The vector steps run in one 1024-thread
// workgroup with fixed-order reductions, so the results do not depend on
// the launch.
#pragma once
#include "kernels.hpp"

namespace rpf {
namespace dev {

// starting point pushed QP_KAPPA of the box width inside, starting duals
// QP_MU0 / slack, primal and dual steps stop QP_TAU of the way to the
// boundary
constexpr double QP_KAPPA = 1e-2;
constexpr double QP_MU0 = 1.0;
constexpr double QP_TAU = 0.995;
constexpr int QP_CHOL_BASE = 16;
constexpr double QP_REG_BASE = 1e-4;
constexpr double QP_REG_UP = 8.0;
constexpr double QP_REG_DOWN = 4.0;
constexpr double QP_REG_MAX = 1e30;
constexpr int QP_NT = 1024;   // threads of the vector-step kernels

// device scalars of the iteration
enum { QS_MAXG = 0, QS_AP, QS_AD, QS_MUC, QS_MUA, QS_MU, QS_ERR, QS_W0, QS_W, QS_WLAST, QS_NSCAL = 12 };
// device words of the iteration (int32)
enum { QF_DONE = 0, QF_ITERS, QF_PIV, QF_RETRY, QF_SKF, QF_SK2, QF_CINFO, QF_FACT, QF_N = 8 };

struct QPVec {
  int nu, m;
  double rho, delta, tol;
  const double* sigma_c;   // [m]
  double* g;               // [n] QP gradient
  double *d, *tl, *tu, *zl, *zu;
  double* sig;             // [n] Sigma = z_l / t_l + z_u / t_u
  double* cs;              // [m] C = rho sigma^2 + Sigma_s
  double* gn;              // [m] rho sigma^2 Sigma_s / C
  double* base;            // [n] -(Hw d + g)
  double *dda, *dzla, *dzua;   // predictor
  double* rhs;             // [n] corrector right-hand side
  double *dd, *dzl, *dzu;  // corrector
  double* ts;              // [m] sigma^2 b_s / C (Schur right-hand side) or sigma^2 d_s (KKT)
  double* rneg;            // [nu] -(b_u + rho J^T ts), input of the Cholesky solve
  double* xu;              // [nu] S^{-1} (b_u + rho J^T ts)
  double* Hd;              // [nu] H d_u
  double* Jv;              // [m] J d_u or J x_u
  double* Jt;              // [nu] J^T ts
  double* qs;              // scalars
  int32_t* done;
  int32_t* iters;
  int32_t* retry;          // the last factorization failed: this slot retries
  int32_t* skF;            // done or retrying
  int32_t* sk2;            // done or the factorization of this slot failed
  int32_t* cinfo;          // info word of this slot's Cholesky (-2: not run)
  int32_t* fact;           // factorization attempts
};

// OP 0: sum, 1: max, 2: min over the workgroup, in a fixed order (wave
// butterflies, then the waves in index order); every thread gets the value
// of lane 0's tree.  sh: LDS of at least blockDim.x / 64 doubles.
template <int OP>
__device__ __forceinline__ double wg_reduce(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = OP == 0 ? v + w : OP == 1 ? fmax(v, w) : fmin(v, w);
  }
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[wv] = v;
  __syncthreads();
  double r = sh[0];
  for (int k = 1; k < nw; ++k) r = OP == 0 ? r + sh[k] : OP == 1 ? fmax(r, sh[k]) : fmin(r, sh[k]);
  return r;
}

// largest step a <= 1 keeping v + a dv >= (1 - tau) v: the candidate of one
// element (infinity when dv >= 0)
__device__ __forceinline__ double step_ratio(double v, double dv, double tau) {
  return dv < 0.0 ? -tau * v / dv : INFINITY;
}

// y[i] = sum_j A[i, j] x[j], A row-major (lda): one wavefront per row,
// four partial sums per lane, combined in a fixed order.
__global__ void __launch_bounds__(256) k_gemv_rows(int rows, int cols, const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ x, double* __restrict__ y,
                                                   const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (i >= rows) return;
  const int lane = threadIdx.x & 63;
  const double* a = A + (size_t)i * lda;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = lane;
  for (; j + 192 < cols; j += 256) {
    s0 += a[j] * x[j];
    s1 += a[j + 64] * x[j + 64];
    s2 += a[j + 128] * x[j + 128];
    s3 += a[j + 192] * x[j + 192];
  }
  for (; j < cols; j += 64) s0 += a[j] * x[j];
  double v = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) y[i] = v;
}

// Partial sums of y = A^T x for a row-major rows x cols matrix: block
// (bx, r) sums rows r*chunk .. (r+1)*chunk - 1 for columns bx*256 + t into
// part[r * cols + col].
__global__ void __launch_bounds__(256) k_gemv_cols_part(int rows, int cols, int chunk, const double* __restrict__ A,
                                                        int64_t lda, const double* __restrict__ x,
                                                        double* __restrict__ part,
                                                        const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  if (c >= cols) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = r0;
  for (; i + 3 < r1; i += 4) {
    s0 += A[(size_t)i * lda + c] * x[i];
    s1 += A[(size_t)(i + 1) * lda + c] * x[i + 1];
    s2 += A[(size_t)(i + 2) * lda + c] * x[i + 2];
    s3 += A[(size_t)(i + 3) * lda + c] * x[i + 3];
  }
  for (; i < r1; ++i) s0 += A[(size_t)i * lda + c] * x[i];
  part[(size_t)blockIdx.y * cols + c] = (s0 + s1) + (s2 + s3);
}

// out[c] = beta * b[c] + alpha * sum_r part[r][c] (r in order); b may be null.
__global__ void k_gemv_cols_sum(int cols, int nparts, const double* __restrict__ part, double alpha,
                                const double* __restrict__ b, double beta, double* __restrict__ out,
                                const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double acc = 0.0;
  for (int r = 0; r < nparts; ++r) acc += part[(size_t)r * cols + c];
  out[c] = alpha * acc + (b ? beta * b[c] : 0.0);
}

// Starting point: bounds of the step lo = w_lo - w, hi = w_hi - w; d the
// origin clipped into [lo + kappa, hi - kappa], kappa = QP_KAPPA (hi - lo);
// slacks and duals; the QP gradient g = (grad, -wc) (wc = D_c (y + rho D_c
// (c - s))) and max |g|; ts = sigma^2 d_s for the first KKT product; the
// first regularisation w0 from max |diag H| (H row-major n_u x n_u).
__global__ void __launch_bounds__(QP_NT) k_qp_init(QPVec Q, const double* __restrict__ u,
                                                   const double* __restrict__ sv, const double* __restrict__ ulo,
                                                   const double* __restrict__ uhi, const double* __restrict__ slo,
                                                   const double* __restrict__ shi, const double* __restrict__ grad,
                                                   const double* __restrict__ wc, const double* __restrict__ H) {
  __shared__ double sh[QP_NT / 64];
  const int n = Q.nu + Q.m;
  double gmax = 0.0, hmax = 0.0;
  for (int i = threadIdx.x; i < Q.nu; i += blockDim.x) hmax = fmax(hmax, fabs(H[(size_t)i * Q.nu + i]));
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const bool isu = i < Q.nu;
    const int k = i - Q.nu;
    const double lo = isu ? ulo[i] - u[i] : slo[k] - sv[k];
    const double hi = isu ? uhi[i] - u[i] : shi[k] - sv[k];
    const double kap = QP_KAPPA * (hi - lo);
    const double d = fmin(fmax(0.0, lo + kap), hi - kap);
    const double tl = d - lo, tu = hi - d;
    Q.d[i] = d;
    Q.tl[i] = tl;
    Q.tu[i] = tu;
    Q.zl[i] = QP_MU0 / tl;
    Q.zu[i] = QP_MU0 / tu;
    const double g = isu ? grad[i] : -wc[k];
    Q.g[i] = g;
    gmax = fmax(gmax, fabs(g));
    if (!isu) {
      const double sc = Q.sigma_c[k];
      Q.ts[k] = sc * sc * d;
    }
  }
  gmax = wg_reduce<1>(gmax, sh);
  hmax = wg_reduce<1>(hmax, sh);
  if (threadIdx.x == 0) {
    Q.qs[QS_MAXG] = gmax;
    Q.qs[QS_W0] = QP_REG_BASE * fmax(1.0, hmax);
    Q.qs[QS_W] = 0.0;
    Q.qs[QS_WLAST] = 0.0;
    Q.done[0] = 0;
    Q.iters[0] = 0;
    Q.retry[0] = 0;
    Q.skF[0] = 0;
    Q.sk2[0] = 0;
    Q.cinfo[0] = -2;
    Q.fact[0] = 0;
  }
}

// start of a slot: skF = done or retrying
__global__ void k_qp_slot(QPVec Q) {
  if (threadIdx.x == 0) Q.skF[0] = (Q.done[0] != 0 || Q.retry[0] != 0) ? 1 : 0;
}

// regularisation of this slot: the Cholesky's info word (-2 = skip when the
// iteration is over), the attempt count
__global__ void k_qp_reg_set(QPVec Q) {
  if (threadIdx.x != 0) return;
  if (Q.done[0] != 0) {
    Q.cinfo[0] = -2;
    return;
  }
  Q.cinfo[0] = 0;
  Q.fact[0] += 1;
}

// Sf = S + w I (row-major n x n), unless the iteration is over
__global__ void k_qp_reg_copy(int n, const double* __restrict__ S, double* __restrict__ Sf, QPVec Q) {
  if (*Q.done) return;
  const double w = Q.qs[QS_W];
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const size_t i = e / n, j = e - i * n;
  Sf[e] = i == j ? S[e] + w : S[e];
}

// after this slot's Cholesky: success keeps w as w_last and lets the solves
// run; failure raises w (w0 if it was 0, else QP_REG_UP w) for a retry in
// the next slot, or ends the iteration past QP_REG_MAX
__global__ void k_qp_reg_check(QPVec Q) {
  if (threadIdx.x != 0) return;
  if (Q.done[0] != 0) {
    Q.sk2[0] = 1;
    return;
  }
  const int ci = Q.cinfo[0];
  if (ci != 0) {
    const double w = Q.qs[QS_W];
    const double wn = w == 0.0 ? Q.qs[QS_W0] : QP_REG_UP * w;
    Q.retry[0] = 1;
    Q.sk2[0] = 1;
    if (wn > QP_REG_MAX) Q.done[0] = QP_CHOL_BASE + (ci > 0 ? ci : 0);
    else Q.qs[QS_W] = wn;
  } else {
    Q.retry[0] = 0;
    Q.sk2[0] = 0;
    Q.qs[QS_WLAST] = Q.qs[QS_W];
  }
}

// KKT test and the Schur data of one iteration.  With Hd = H d_u,
// Jv = J d_u, Jt = J^T (sigma^2 d_s):
//   q = Hw d = (Hd + delta d_u - rho Jt, rho sigma^2 (d_s - Jv)),
//   r = q + g - z_l + z_u, base = -(q + g),
//   err = max(max|r| / (1 + max|g|), max(t_l z_l), max(t_u z_u)).
// err < tol sets done = 1 (a non-finite r sets 2).  Unless done, or when
// final != 0, then Sigma, C, the curvature weights gn and the predictor's
// Schur right-hand side ts = sigma^2 base_s / C.
__global__ void __launch_bounds__(QP_NT) k_qp_kkt(QPVec Q, int final_check) {
  if (*Q.skF) return;
  __shared__ double sh[QP_NT / 64];
  const int n = Q.nu + Q.m;
  double amax = 0.0, cmax = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const bool isu = i < Q.nu;
    const int k = i - Q.nu;
    double q;
    if (isu) {
      q = Q.Hd[i] + Q.delta * Q.d[i] - Q.rho * Q.Jt[i];
    } else {
      const double sc = Q.sigma_c[k];
      q = Q.rho * (sc * sc) * (Q.d[i] - Q.Jv[k]);
    }
    const double qg = q + Q.g[i];
    const double zl = Q.zl[i], zu = Q.zu[i];
    const double r = qg - zl + zu;
    Q.base[i] = -qg;
    amax = fmax(amax, fabs(r));
    cmax = fmax(cmax, fmax(Q.tl[i] * zl, Q.tu[i] * zu));
    if (!isfinite(r)) bad = 1.0;
  }
  amax = wg_reduce<1>(amax, sh);
  cmax = wg_reduce<1>(cmax, sh);
  bad = wg_reduce<1>(bad, sh);
  const double err = fmax(amax / (1.0 + Q.qs[QS_MAXG]), cmax);
  const bool stop = bad > 0.0 || err < Q.tol;
  if (threadIdx.x == 0) {
    Q.qs[QS_ERR] = bad > 0.0 ? NAN : err;
    if (bad > 0.0) Q.done[0] = 2;
    else if (err < Q.tol) Q.done[0] = 1;
    if (stop) Q.skF[0] = 1;
    if (!stop && !final_check) {
      // first regularisation of the iteration
      const double wl = Q.qs[QS_WLAST];
      Q.qs[QS_W] = wl == 0.0 ? 0.0 : fmax(Q.qs[QS_W0], wl / QP_REG_DOWN);
    }
  }
  if (stop || final_check) return;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double sg = Q.zl[i] / Q.tl[i] + Q.zu[i] / Q.tu[i];
    Q.sig[i] = sg;
    if (i >= Q.nu) {
      const int k = i - Q.nu;
      const double sc = Q.sigma_c[k];
      const double r2 = Q.rho * (sc * sc);
      const double c = r2 + sg;
      Q.cs[k] = c;
      Q.gn[k] = r2 * sg / c;
      Q.ts[k] = sc * sc * Q.base[i] / c;
    }
  }
}

// Predictor (affine) step from the Schur solution of (Hw + Sigma) dda = base
// (xu, Jv = J xu): the dual steps, the largest steps to the boundary ap, ad,
// the complementarity mu_c and the one the affine step would reach mu_a,
// the centring target mu = (mu_a / mu_c)^3 mu_c, and the corrector's
// right-hand side rhs = base + r_l / t_l - r_u / t_u with r_l = mu - dda
// dz_la, r_u = mu + dda dz_ua (ts = sigma^2 rhs_s / C for its Schur solve).
__global__ void __launch_bounds__(QP_NT) k_qp_pred(QPVec Q) {
  const int k2 = *Q.sk2;
  if (k2 < 0 && threadIdx.x == 0 && Q.done[0] == 0) Q.done[0] = -1;   // a solve gave up waiting
  if (k2) return;
  __shared__ double sh[QP_NT / 64];
  const int n = Q.nu + Q.m;
  double ap = INFINITY, ad = INFINITY, cs = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const bool isu = i < Q.nu;
    const int k = i - Q.nu;
    double dx;
    if (isu) {
      dx = Q.xu[i];
    } else {
      const double sc = Q.sigma_c[k];
      dx = (Q.base[i] + Q.rho * (sc * sc) * Q.Jv[k]) / Q.cs[k];
    }
    const double tl = Q.tl[i], tu = Q.tu[i], zl = Q.zl[i], zu = Q.zu[i];
    const double dzl = -zl - (zl / tl) * dx;
    const double dzu = -zu + (zu / tu) * dx;
    Q.dda[i] = dx;
    Q.dzla[i] = dzl;
    Q.dzua[i] = dzu;
    ap = fmin(ap, fmin(step_ratio(tl, dx, 1.0), step_ratio(tu, -dx, 1.0)));
    ad = fmin(ad, fmin(step_ratio(zl, dzl, 1.0), step_ratio(zu, dzu, 1.0)));
    cs += tl * zl + tu * zu;
  }
  ap = fmin(1.0, wg_reduce<2>(ap, sh));
  ad = fmin(1.0, wg_reduce<2>(ad, sh));
  const double muc = wg_reduce<0>(cs, sh) / (2.0 * n);
  double ms = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double dx = Q.dda[i];
    ms += (Q.tl[i] + ap * dx) * (Q.zl[i] + ad * Q.dzla[i]) + (Q.tu[i] - ap * dx) * (Q.zu[i] + ad * Q.dzua[i]);
  }
  const double mua = wg_reduce<0>(ms, sh) / (2.0 * n);
  const double ratio = mua / muc;
  const double mu = ratio * ratio * ratio * muc;
  if (threadIdx.x == 0) {
    Q.qs[QS_MUC] = muc;
    Q.qs[QS_MUA] = mua;
    Q.qs[QS_MU] = mu;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double dx = Q.dda[i];
    const double rl = mu - dx * Q.dzla[i];
    const double ru = mu + dx * Q.dzua[i];
    const double b = Q.base[i] + rl / Q.tl[i] - ru / Q.tu[i];
    Q.rhs[i] = b;
    if (i >= Q.nu) {
      const int k = i - Q.nu;
      const double sc = Q.sigma_c[k];
      Q.ts[k] = sc * sc * b / Q.cs[k];
    }
  }
}

// Corrector step from the Schur solution of (Hw + Sigma) dd = rhs (xu,
// Jv = J xu): dz_l = r_l / t_l - z_l - z_l / t_l dd, dz_u = r_u / t_u - z_u
// + z_u / t_u dd, steps QP_TAU of the way to the boundary, then the update
// of d, t_l, t_u, z_l, z_u and ts = sigma^2 d_s for the next KKT product.
__global__ void __launch_bounds__(QP_NT) k_qp_corr(QPVec Q) {
  const int k2 = *Q.sk2;
  if (k2 < 0 && threadIdx.x == 0 && Q.done[0] == 0) Q.done[0] = -1;
  if (k2) return;
  __shared__ double sh[QP_NT / 64];
  const int n = Q.nu + Q.m;
  const double mu = Q.qs[QS_MU];
  double ap = INFINITY, ad = INFINITY;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const bool isu = i < Q.nu;
    const int k = i - Q.nu;
    double dx;
    if (isu) {
      dx = Q.xu[i];
    } else {
      const double sc = Q.sigma_c[k];
      dx = (Q.rhs[i] + Q.rho * (sc * sc) * Q.Jv[k]) / Q.cs[k];
    }
    const double tl = Q.tl[i], tu = Q.tu[i], zl = Q.zl[i], zu = Q.zu[i];
    const double da = Q.dda[i];
    const double rl = mu - da * Q.dzla[i];
    const double ru = mu + da * Q.dzua[i];
    const double dzl = rl / tl - zl - (zl / tl) * dx;
    const double dzu = ru / tu - zu + (zu / tu) * dx;
    Q.dd[i] = dx;
    Q.dzl[i] = dzl;
    Q.dzu[i] = dzu;
    ap = fmin(ap, fmin(step_ratio(tl, dx, QP_TAU), step_ratio(tu, -dx, QP_TAU)));
    ad = fmin(ad, fmin(step_ratio(zl, dzl, QP_TAU), step_ratio(zu, dzu, QP_TAU)));
  }
  ap = fmin(1.0, wg_reduce<2>(ap, sh));
  ad = fmin(1.0, wg_reduce<2>(ad, sh));
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double dx = Q.dd[i];
    const double d = Q.d[i] + ap * dx;
    Q.d[i] = d;
    Q.tl[i] = Q.tl[i] + ap * dx;
    Q.tu[i] = Q.tu[i] - ap * dx;
    Q.zl[i] = Q.zl[i] + ad * Q.dzl[i];
    Q.zu[i] = Q.zu[i] + ad * Q.dzu[i];
    if (i >= Q.nu) {
      const double sc = Q.sigma_c[i - Q.nu];
      Q.ts[i - Q.nu] = sc * sc * d;
    }
  }
  if (threadIdx.x == 0) {
    Q.qs[QS_AP] = ap;
    Q.qs[QS_AD] = ad;
    Q.iters[0] += 1;
  }
}

// status = {iterations, converged, Cholesky info of S (1-based column of
// the last failed Cholesky once the regularisation gave up, -1 solve wait
// expired, 0), done word, (tiny pivot word, copied by the caller),
// factorization attempts}; kkt = last KKT error, wreg = last successful
// regularisation.
__global__ void k_qp_status(const int32_t* __restrict__ f, const double* __restrict__ qs,
                            int32_t* __restrict__ status, double* __restrict__ kkt, double* __restrict__ wreg) {
  const int dn = f[QF_DONE];
  status[0] = f[QF_ITERS];
  status[1] = dn == 1 ? 1 : 0;
  status[2] = dn >= QP_CHOL_BASE ? dn - QP_CHOL_BASE : (dn < 0 ? -1 : 0);
  status[3] = dn;
  status[4] = f[QF_PIV];
  status[5] = f[QF_FACT];
  if (kkt) kkt[0] = qs[QS_ERR];
  if (wreg) wreg[0] = qs[QS_WLAST];
}

// Scalars of the static OPF driver (one workgroup): out[0] = the
// projected-gradient measure ||w - clip(w - g, lo, hi)||_inf of w = (u, s)
// with the QP gradient g, out[1] = g . d with the QP step d.
__global__ void __launch_bounds__(QP_NT) k_static_pg(int nu, int m, const double* __restrict__ u,
                                                     const double* __restrict__ sv, const double* __restrict__ ulo,
                                                     const double* __restrict__ uhi, const double* __restrict__ slo,
                                                     const double* __restrict__ shi, const double* __restrict__ g,
                                                     const double* __restrict__ d, double* __restrict__ out) {
  __shared__ double sh[QP_NT / 64];
  const int n = nu + m;
  double pg = 0.0, sl = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const bool isu = i < nu;
    const double w = isu ? u[i] : sv[i - nu];
    const double lo = isu ? ulo[i] : slo[i - nu];
    const double hi = isu ? uhi[i] : shi[i - nu];
    pg = fmax(pg, fabs(w - fmin(fmax(w - g[i], lo), hi)));
    sl += g[i] * d[i];
  }
  pg = wg_reduce<1>(pg, sh);
  sl = wg_reduce<0>(sl, sh);
  if (threadIdx.x == 0) {
    out[0] = pg;
    out[1] = sl;
  }
}

// out[0] = ||c - s||_inf over the m constraints (one workgroup)
__global__ void __launch_bounds__(QP_NT) k_static_theta(int m, const double* __restrict__ c,
                                                        const double* __restrict__ sv, double* __restrict__ out) {
  __shared__ double sh[QP_NT / 64];
  double th = 0.0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) th = fmax(th, fabs(c[k] - sv[k]));
  th = wg_reduce<1>(th, sh);
  if (threadIdx.x == 0) out[0] = th;
}

}  // namespace dev
}  // namespace rpf
