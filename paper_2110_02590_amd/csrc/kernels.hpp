// Device kernels of the reduced-space hot path (gfx950, wave64, FP64).
//
// Data layout: state vectors in the internal (fill-reducing) order, controls
// in the paper's order; batches of vectors are row-major [n x ld] blocks so
// that the lanes of a wavefront run over directions (columns) and every row
// access is contiguous.  All reductions are deterministic (fixed gather
// orders, no floating-point atomics).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "presolve.hpp"

namespace rpf {
namespace dev {

using rpf::RECW;
using rpf::WREC;
constexpr int CB = 64;  // dense block width
using rpf::TAIL_MAX;   // leading dimension of the dense pack tails
typedef double dbl4 __attribute__((ext_vector_type(4)));

// Staging through LDS issues all of a thread's loads before its first
// store: a loop that stores each loaded value would wait for memory once
// per iteration.  Addresses are clamped into the source block, so every
// load is in bounds.

// CB x CB tile: element (r, c) = src[r * ld + c] for r < nr, c < nc (nr,
// nc >= 1); elsewhere diag_pad on the diagonal and 0 off it.  TRANS stores
// dst[c][r].  NT = threads of the block.
template <int NT, bool TRANS = false>
__device__ __forceinline__ void stage_tile(double (*dst)[CB + 1], const double* __restrict__ src, size_t ld, int nr, int nc,
                                  double diag_pad) {
  constexpr int PER = CB * CB / NT;
  double v[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = threadIdx.x + m * NT, r = e >> 6, c = e & 63;
    const double g = src[(size_t)min(r, nr - 1) * ld + min(c, nc - 1)];
    v[m] = (r < nr && c < nc) ? g : (r == c ? diag_pad : 0.0);
  }
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = threadIdx.x + m * NT, r = e >> 6, c = e & 63;
    if (TRANS) dst[c][r] = v[m];
    else dst[r][c] = v[m];
  }
}

// Two CB x CB tiles as stage_tile (the second stored transposed with
// TRANS2), every load of both issued before the first store: one memory
// round trip for the pair.
template <int NT, bool TRANS2>
__device__ __forceinline__ void stage_tile_pair(double (*d1)[CB + 1], const double* __restrict__ s1, int nr1, int nc1,
                                                double (*d2)[CB + 1], const double* __restrict__ s2, int nr2, int nc2,
                                                size_t ld, double diag_pad) {
  constexpr int PER = CB * CB / NT;
  double v1[PER], v2[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = threadIdx.x + m * NT, r = e >> 6, c = e & 63;
    v1[m] = s1[(size_t)min(r, nr1 - 1) * ld + min(c, nc1 - 1)];
    v2[m] = s2[(size_t)min(r, nr2 - 1) * ld + min(c, nc2 - 1)];
  }
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = threadIdx.x + m * NT, r = e >> 6, c = e & 63;
    const double pad = r == c ? diag_pad : 0.0;
    d1[r][c] = (r < nr1 && c < nc1) ? v1[m] : pad;
    const double w2 = (r < nr2 && c < nc2) ? v2[m] : pad;
    if (TRANS2) d2[c][r] = w2;
    else d2[r][c] = w2;
  }
}

// Workgroup barrier for kernels whose threads communicate only through LDS:
// waits for the thread's LDS operations, not for its global loads, so
// prefetched global data can stay in flight across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// dst[e] = src[e] for e < n, eight loads in flight per thread.
template <class T>
__device__ __forceinline__ void stage_1d(T* dst, const T* __restrict__ src, int n) {
  const int nt = blockDim.x;
  for (int e0 = threadIdx.x; e0 < n; e0 += 8 * nt) {
    T v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = src[min(e0 + m * nt, n - 1)];
#pragma unroll
    for (int m = 0; m < 8; ++m)
      if (e0 + m * nt < n) dst[e0 + m * nt] = v[m];
  }
}

// ------------------------------------------------------------------ helpers
__global__ void k_permute_gather(int n, const int32_t* __restrict__ idx, const double* __restrict__ src,
                                 double* __restrict__ dst,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

__global__ void k_permute_scatter(int n, const int32_t* __restrict__ idx, const double* __restrict__ src,
                                  double* __restrict__ dst,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = src[i];
}

// out[i] = base[i] + sum_{j in [ptr[i], ptr[i+1])} in[src[j]]
__global__ void k_gather_sum(int n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
                             const double* __restrict__ in, const double* __restrict__ base,
                             double* __restrict__ out,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = base ? base[i] : 0.0;
  for (int j = ptr[i]; j < ptr[i + 1]; ++j) acc += in[src[j]];
  out[i] = acc;
}

// out[p] = in[srcpos[p]]
__global__ void k_gather_pos(int n, const int32_t* __restrict__ srcpos, const double* __restrict__ in,
                             double* __restrict__ out,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[srcpos[i]];
}

// ------------------------------------------------------------- bus state
__global__ void k_bus_state(int nb, int nx, const int32_t* __restrict__ th_var,
                            const int32_t* __restrict__ v_var, const double* __restrict__ xi,
                            const double* __restrict__ u, double* __restrict__ th, double* __restrict__ vm,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int a = th_var[i];
  th[i] = a >= 0 ? xi[a] : 0.0;
  int b = v_var[i];
  vm[i] = b < nx ? xi[b] : u[b - nx];
}

// --------------------------------------------------------- branch records
// One thread per branch: flows at both ends of the pi model and their
// partial derivatives with respect to (theta_f, theta_t, v_f, v_t).
// Each end flow is v_o^2 K_o + v_f v_t T(theta_f - theta_t) with T'' = -T.
__global__ void k_branch_eval(int nl, const int32_t* __restrict__ bf, const int32_t* __restrict__ bt,
                              const double* __restrict__ br, const double* __restrict__ bx,
                              const double* __restrict__ bb, const double* __restrict__ th,
                              const double* __restrict__ vm, double* __restrict__ rec,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  int f = bf[l], t = bt[l];
  double r = br[l], x = bx[l], bsh = 0.5 * bb[l];
  double z2 = r * r + x * x;
  double gs = r / z2, bs = -x / z2;
  // self (own) admittance Y_oo = gs + j(bs + b/2); mutual Y_ft = Y_tf = -gs - j bs
  double Goo = gs, Boo = bs + bsh, Gm = -gs, Bm = -bs;
  double vf = vm[f], vt = vm[t];
  double d = th[f] - th[t];
  double sn, cs;
  sincos(d, &sn, &cs);
  double vv = vf * vt;
  // from end: A = Gm cos + Bm sin, C = Gm sin - Bm cos; A' = -C, C' = A
  double Af = Gm * cs + Bm * sn, Cf = Gm * sn - Bm * cs;
  // to end:   A = Gm cos - Bm sin, C = -Gm sin - Bm cos; A' = C, C' = -A
  double At = Gm * cs - Bm * sn, Ct = -Gm * sn - Bm * cs;
  double* o = rec + (size_t)l * RECW;
  o[0] = vf * vf * Goo + vv * Af;
  o[1] = -vf * vf * Boo + vv * Cf;
  o[2] = vt * vt * Goo + vv * At;
  o[3] = -vt * vt * Boo + vv * Ct;
  // P_f: T = Af, T' = -Cf, own f, K = Goo
  o[4] = -vv * Cf;
  o[5] = vv * Cf;
  o[6] = vt * Af + 2.0 * vf * Goo;
  o[7] = vf * Af;
  // Q_f: T = Cf, T' = Af, own f, K = -Boo
  o[8] = vv * Af;
  o[9] = -vv * Af;
  o[10] = vt * Cf - 2.0 * vf * Boo;
  o[11] = vf * Cf;
  // P_t: T = At, T' = Ct, own t, K = Goo
  o[12] = vv * Ct;
  o[13] = -vv * Ct;
  o[14] = vt * At;
  o[15] = vf * At + 2.0 * vt * Goo;
  // Q_t: T = Ct, T' = -At, own t, K = -Boo
  o[16] = -vv * At;
  o[17] = vv * At;
  o[18] = vt * Ct;
  o[19] = vf * Ct - 2.0 * vt * Boo;
}

// ------------------------------------------------------------- residual
// g[row] = sum of branch-end flows at the row's bus + load - p_pv, and the
// per-block partial sums of g^2.
__global__ void k_residual(int nx, const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
                           const double* __restrict__ rec, const int32_t* __restrict__ row_bus,
                           const int32_t* __restrict__ row_isq, const int32_t* __restrict__ row_pvar,
                           const double* __restrict__ pd, const double* __restrict__ qd,
                           const double* __restrict__ u, double* __restrict__ g,
                           double* __restrict__ partial,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double red[256];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < nx) {
    double acc = 0.0;
    for (int j = ptr[i]; j < ptr[i + 1]; ++j) acc += rec[src[j]];
    int b = row_bus[i];
    acc += row_isq[i] ? qd[b] : pd[b];
    int pv = row_pvar[i];
    if (pv >= 0) acc -= u[pv];
    g[i] = acc;
    v = acc * acc;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Single-block deterministic sum of `n` values; optionally sqrt.  Also sets
// done[0] = (result < tol) when done is given.
__global__ void k_reduce_final(int n, const double* __restrict__ in, double* __restrict__ out,
                               int take_sqrt, double tol, int32_t* __restrict__ done,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double red[1024];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += in[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double r = take_sqrt ? sqrt(red[0]) : red[0];
    out[0] = r;
    // done: 1 converged, 2 non-finite residual (diverged), 0 otherwise
    if (done) done[0] = (r < tol) ? 1 : (isfinite(r) ? 0 : 2);
  }
}

// lane s's 64-bit value (s uniform)
__device__ __forceinline__ int64_t readlane64(int64_t v, int s) {
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(v & 0xffffffff), s);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), s);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// lane s's double (s uniform)
__device__ __forceinline__ double readlane_f64(double v, int s) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), s);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), s);
  return __hiloint2double(hi, lo);
}

// ----------------------------------------------------- LU refactorization
// Row-by-row (up-looking) elimination on the static pattern, one wavefront
// per row with the row staged in LDS: for each L entry (i, k), k ascending,
// l_ik = a_ik / u_kk and a_ij -= l_ik u_kj for the U entries of row k
// (target positions precomputed).  Only L entries in [ptr[i], pend) are
// eliminated.  Rows k are final when row i starts, so their data (pivot
// reciprocal rdg[k] = 1 / u_kk, U values, targets) are loaded ahead: the
// metadata of 64 steps at once, the values and targets two steps ahead;
// only the row's own entries in LDS form the dependency chain.  The
// finished row stores 1 / u_ii in rdg[i].  With check, a pivot
// |u_ii| <= pivtol max_j |a_ij| records row + 1 in status[0].
__device__ __forceinline__ void rf_row(int i, int pend, bool check, const int32_t* __restrict__ ptr,
                              const int32_t* __restrict__ col, const int32_t* __restrict__ diag,
                              const int64_t* __restrict__ upd_ptr, const int32_t* __restrict__ upd_tgt,
                              double* __restrict__ a, double* __restrict__ rdg, double* __restrict__ w,
                              double pivtol, int32_t* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int p0 = ptr[i], pdg = diag[i], p1 = ptr[i + 1];
  double amax = 0.0;
  for (int q = lane; q < p1 - p0; q += 64) {
    double v = a[p0 + q];
    w[q] = v;
    amax = fmax(amax, fabs(v));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // Steps in windows of 64: lane j loads step w0 + j's metadata (column k,
  // U row start diag[k] + 1, 1 / u_kk, update range) in one batch; a step
  // reads it by readlane.  Its U values and update targets are loaded two
  // steps ahead, unconditionally from clamped addresses (upd_tgt is padded
  // past its end), since they do not depend on the row being eliminated.
  for (int w0 = p0; w0 < pend; w0 += 64) {
    const int nw = min(64, pend - w0);
    const int pm = w0 + min(lane, nw - 1);
    const int km = col[pm];
    const int m_dk = diag[km];
    const double m_rk = rdg[km];
    const int64_t m_u0 = upd_ptr[pm];
    const int m_nu = (int)(upd_ptr[pm + 1] - m_u0);
    auto fetch = [&](int st, int& tg, double& av) {
      const int64_t u0 = readlane64(m_u0, st);
      const int nu = __builtin_amdgcn_readlane(m_nu, st);
      const int dk = __builtin_amdgcn_readlane(m_dk, st);
      const int q = min(lane, max(nu - 1, 0));
      tg = upd_tgt[u0 + q];
      av = a[dk + (nu > 0 ? 1 + q : 0)];
    };
    auto step = [&](int st, int tg, double av) {
      const int p = w0 + st;
      const int nu = __builtin_amdgcn_readlane(m_nu, st);
      const double l = w[p - p0] * readlane_f64(m_rk, st);
      if (lane < nu) w[tg - p0] -= l * av;
      if (nu > 64) {
        const int64_t u0 = readlane64(m_u0, st);
        const int dk = __builtin_amdgcn_readlane(m_dk, st);
        for (int t = lane + 64; t < nu; t += 64) w[upd_tgt[u0 + t] - p0] -= l * a[dk + 1 + t];
      }
      if (lane == 0) w[p - p0] = l;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    int tgA, tgB;
    double avA, avB;
    fetch(0, tgA, avA);
    fetch(min(1, nw - 1), tgB, avB);
    for (int st = 0; st < nw; st += 2) {
      step(st, tgA, avA);
      fetch(min(st + 2, nw - 1), tgA, avA);
      if (st + 1 < nw) step(st + 1, tgB, avB);
      fetch(min(st + 3, nw - 1), tgB, avB);
    }
  }
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  for (int q = lane; q < p1 - p0; q += 64) a[p0 + q] = w[q];
  if (lane == 0) {
    const double piv = w[pdg - p0];
    rdg[i] = 1.0 / piv;
    if (check && !(fabs(piv) > pivtol * amax)) atomicCAS(status, 0, i + 1);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Packs of independent subtrees: one workgroup per pack, its forward levels
// separated by workgroup barriers, one wavefront per row.
__global__ void k_rf_pack(const int32_t* __restrict__ flev, const int32_t* __restrict__ flev_off,
                          const int32_t* __restrict__ frows, const int32_t* __restrict__ ptr,
                          const int32_t* __restrict__ col, const int32_t* __restrict__ diag,
                          const int64_t* __restrict__ upd_ptr, const int32_t* __restrict__ upd_tgt,
                          double* __restrict__ a, double* __restrict__ rdg, int maxrow, double pivtol,
                          int32_t* __restrict__ status, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ double lds[];
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  double* w = lds + (size_t)wave * maxrow;
  const int q = blockIdx.x;
  for (int lv = flev_off[q]; lv < flev_off[q + 1]; ++lv) {
    for (int r = flev[lv] + wave; r < flev[lv + 1]; r += nwave) {
      const int i = frows[r];
      rf_row(i, diag[i], true, ptr, col, diag, upd_ptr, upd_tgt, a, rdg, w, pivtol, status);
    }
    __syncthreads();
  }
}


// v of the lane that the DPP control CTRL selects (every lane active)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// v(lane) + v(lane xor 16) and v(lane) + v(lane xor 32), in registers: the
// permlane swaps exchange alternate 16-lane rows (32-lane halves) of their
// two operands; with v in both, the two results hold v of the lane and of
// its partner, in one order or the other (the sum is the same either way)
__device__ __forceinline__ double sum_xor16(double v) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double sum_xor32(double v) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// Sum over aligned groups of G consecutive lanes (G a power of two, at most
// 64, uniform); every lane of a group receives the group's sum.  Within
// rows of 16 lanes by DPP (quad permutations, then the half-row and row
// mirrors, each pairing a lane with one holding the other half's partial
// sum), across rows by permlane swaps.  Every lane must be active.
__device__ __forceinline__ double group_sum(double v, int G) {
  if (G >= 2) v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  if (G >= 4) v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  if (G >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
  if (G >= 16) v += dpp_f64<0x140>(v);  // row_mirror
  if (G >= 32) v = sum_xor16(v);
  if (G >= 64) v = sum_xor32(v);
  return v;
}

// Elimination steps between the load of a step's update targets and the
// step itself in the LDS-resident refactorization.
constexpr int RF_AHEAD = 4;

// Packs with their LU values resident in LDS: one workgroup (16
// wavefronts) per pack, forward levels separated by barriers, one
// wavefront per row, eliminating in place in LDS.  The metadata of up to
// 64 elimination steps of a row (pivot column, U-row start, update range)
// is loaded at once, lane s holding step s, and broadcast by readlane --
// for a wavefront's next row while it works on the current one; the
// update targets of step s + RF_AHEAD are loaded during step s.
// Reciprocal pivots of finished rows go to LDS and to rdg.  upd_tgt must
// hold 64 readable entries past its end, ent and entu0 one entry past
// theirs.  LDS: values of the pack's CSR rows [seg] | 1 / u_ii [nr] | with
// RECS_LDS, the program's row records [nprog] (16-byte aligned; otherwise
// they are read from global memory).
//
// Dense tails (toff non-null; flev the batched forward program): the last
// level holds the pack's tail rows T (in the order of trows), which
// eliminate only their columns outside T there and keep their pivots open.
// Then the T x T block is finished right-looking, one tail pivot k at a
// time (one barrier per pivot): every L entry (i, k) of a later tail row
// (tlrec[tl_ptr[g] .. tl_ptr[g + 1]), g the pivot's tail index) takes l =
// a_ik / u_kk and updates row i's targets of row k's U entries (tail and
// top columns), the rows in parallel.
// Static records (built on the host): rowrec per program position {row,
// diagonal position, first and end entry of its elimination list}, staged
// in LDS; ent per list entry {LU position, pivot column, U-row start of the
// pivot row, update count} with entu0 its first update; tlrec per tail
// entry {LU position, U-row start, update count, first update}.
template <bool RECS_LDS>
__global__ void __launch_bounds__(1024) k_rf_pack_lds(const int32_t* __restrict__ pack_ptr,
                                                      const int32_t* __restrict__ flev,
                                                      const int32_t* __restrict__ flev_off,
                                                      const int4* __restrict__ rowrec,
                                                      const int32_t* __restrict__ ptr,
                                                      const int4* __restrict__ ent,
                                                      const int32_t* __restrict__ entu0,
                                                      const int32_t* __restrict__ upd_tgt,
                                                      double* __restrict__ a, double* __restrict__ rdg,
                                                      double pivtol, int32_t* __restrict__ status,
                                                      const int32_t* __restrict__ skip,
                                                      const int32_t* __restrict__ toff,
                                                      const int16_t* __restrict__ trows,
                                                      const int32_t* __restrict__ tl_ptr,
                                                      const int4* __restrict__ tlrec) {
  if (skip && *skip) return;
  extern __shared__ double sv[];
  const int q = blockIdx.x;
  const int r0 = pack_ptr[q], nr = pack_ptr[q + 1] - r0;
  const int gp0 = ptr[r0], seg = ptr[r0 + nr] - gp0;
  const int lv0 = flev_off[q], lv1 = flev_off[q + 1];
  const int base = flev[lv0], nprog = flev[lv1] - base;
  double* srd = sv + seg;
  int4* srec_l = reinterpret_cast<int4*>((reinterpret_cast<uintptr_t>(srd + nr) + 15) & ~uintptr_t(15));
  const int4* srec = RECS_LDS ? srec_l : rowrec + base;
  const int t = threadIdx.x;
  stage_1d(sv, a + gp0, seg);
  if (RECS_LDS)
    for (int k = t; k < nprog; k += blockDim.x) srec_l[k] = rowrec[base + k];
  __syncthreads();
  // max |a_ij| of each row before elimination, for the pivot test, kept in
  // the row's reciprocal-pivot slot until the row is finished (no step
  // reads a slot before its row is done)
  for (int r = t; r < nr; r += blockDim.x) {
    const int p0 = ptr[r0 + r] - gp0, p1 = ptr[r0 + r + 1] - gp0;
    double m0 = 0.0, m1 = 0.0;
    int e = p0;
    for (; e + 1 < p1; e += 2) {
      m0 = fmax(m0, fabs(sv[e]));
      m1 = fmax(m1, fabs(sv[e + 1]));
    }
    if (e < p1) m0 = fmax(m0, fabs(sv[e]));
    srd[r] = fmax(m0, m1);
  }
  __syncthreads();
  const int wave = t >> 6, lane = t & 63, nwave = blockDim.x >> 6;
  const int tq = toff ? toff[q] : 0, nT = toff ? toff[q + 1] - tq : 0;
  // a row's step metadata (lane s: step s of its first 64) is loaded one
  // row ahead: during row rr the wavefront's next row's records are in
  // flight
  int4 nE = make_int4(0, 0, 0, 0);
  int nU = 0;
  auto fetch_row = [&](int rr) {
    const int4 R = srec[rr - base];
    const int e0 = R.z, nw = min(64, R.w - R.z);
    const int e = e0 + (lane < nw ? lane : 0);
    nE = ent[e];
    nU = entu0[e];
  };
  for (int lv = lv0; lv < lv1; ++lv) {
    const bool tail = nT > 0 && lv == lv1 - 1;   // the tail rows: pivots stay open
    const int rend = flev[lv + 1];
    int rr = flev[lv] + wave;
    if (rr < rend) fetch_row(rr);
    for (; rr < rend; rr += nwave) {
      // the row record is the same in every lane: keep it scalar
      const int4 R = srec[rr - base];
      const int i = __builtin_amdgcn_readfirstlane(R.x);
      const int pdg = __builtin_amdgcn_readfirstlane(R.y);
      const int e0 = __builtin_amdgcn_readfirstlane(R.z);
      const int e1 = __builtin_amdgcn_readfirstlane(R.w);
      int4 cE = nE;
      int cU = nU;
      if (rr + nwave < rend) fetch_row(rr + nwave);
      for (int w0 = e0; w0 < e1; w0 += 64) {
        const int nw = min(64, e1 - w0);
        if (w0 != e0) {
          const int e = w0 + (lane < nw ? lane : 0);
          cE = ent[e];
          cU = entu0[e];
        }
        const int m_p = lane < nw ? cE.x : 0;
        const int m_k = lane < nw ? cE.y : 0;
        const int m_us = lane < nw ? cE.z : 0;
        const int m_nu = lane < nw ? cE.w : 0;
        const int m_u0 = lane < nw ? cU : 0;
        // targets of step s live in tg[s mod RF_AHEAD]; the load for step
        // s + RF_AHEAD is issued during step s into the same register:
        // unconditional loads (upd_tgt is padded past its end), so the
        // compiler can count them and wait only for the oldest one
        auto fetch_tg = [&](int st) -> int {
          const int u = __builtin_amdgcn_readlane(m_u0, st);
          return upd_tgt[u + (lane < __builtin_amdgcn_readlane(m_nu, st) ? lane : 0)];
        };
        // the U entry and the target's current value are read with clamped
        // addresses (no branch around the reads; a wavefront's LDS
        // operations complete in order, so they see every earlier step's
        // stores); only the store is predicated
        auto step = [&](int st, int tgabs) {
          const int k = __builtin_amdgcn_readlane(m_k, st);
          const int us = __builtin_amdgcn_readlane(m_us, st) - gp0;
          const int nu = __builtin_amdgcn_readlane(m_nu, st);
          const int pl = __builtin_amdgcn_readlane(m_p, st) - gp0;
          const bool on = lane < nu;
          const double av = sv[us + (on ? lane : 0)];
          const double cur = sv[on ? tgabs - gp0 : pl];
          const double l = sv[pl] * srd[k - r0];
          if (on) sv[tgabs - gp0] = cur - l * av;
          if (nu > 64) {
            const int u0 = __builtin_amdgcn_readlane(m_u0, st);
            for (int tt = lane + 64; tt < nu; tt += 64) sv[upd_tgt[u0 + tt] - gp0] -= l * sv[us + tt];
          }
          if (lane == 0) sv[pl] = l;
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        };
        int tg[RF_AHEAD];
#pragma unroll
        for (int d = 0; d < RF_AHEAD; ++d) tg[d] = fetch_tg(min(d, nw - 1));
        for (int st = 0; st < nw; st += RF_AHEAD) {
#pragma unroll
          for (int d = 0; d < RF_AHEAD; ++d) {
            if (st + d < nw) step(st + d, tg[d]);
            tg[d] = fetch_tg(min(st + d + RF_AHEAD, nw - 1));
          }
        }
      }
      if (lane == 0 && !tail) {
        const double amax = srd[i - r0];
        const double piv = sv[pdg - gp0];
        const double rp = 1.0 / piv;
        srd[i - r0] = rp;
        rdg[i] = rp;
        if (!(fabs(piv) > pivtol * amax)) atomicCAS(status, 0, i + 1);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    lds_barrier();
  }
  // the tail block, right-looking over its pivots: entry c of pivot g's
  // list (wavefront c mod 16) has its record {LU position, U-row start,
  // update count, first update} and its update targets loaded during the
  // previous pivot
  int4 tR = make_int4(0, 0, 0, 0);
  int tT = 0;
  auto fetch_tail = [&](int b) {
    const int g = tq + b;
    const int c = tl_ptr[g] + wave;
    if (c < tl_ptr[g + 1]) {
      tR = tlrec[c];
      tT = upd_tgt[tR.w + (lane < tR.z ? lane : 0)];
    }
  };
  const int tbase = flev[lv1 - 1] - base;
  if (nT > 0) fetch_tail(0);
  for (int b = 0; b < nT; ++b) {
    // the tail rows are the program's last level, in the order of trows
    const int4 KR = srec[tbase + b];
    const int k = __builtin_amdgcn_readfirstlane(KR.x);
    const int pk = __builtin_amdgcn_readfirstlane(KR.y);
    const int g = tq + b;
    const int c0 = tl_ptr[g], c1 = tl_ptr[g + 1];
    const int4 cR = tR;
    const int cT = tT;
    if (b + 1 < nT) fetch_tail(b + 1);
    const double piv = sv[pk - gp0];   // final: every earlier pivot has updated row k
    if (t == 0) {
      const double rp = 1.0 / piv;
      rdg[k] = rp;
      if (!(fabs(piv) > pivtol * srd[k - r0])) atomicCAS(status, 0, k + 1);
    }
    const double rp = 1.0 / piv;
    for (int c = c0 + wave; c < c1; c += nwave) {
      int4 R = cR;
      int tg = cT;
      if (c != c0 + wave) {
        R = tlrec[c];
        tg = upd_tgt[R.w + (lane < R.z ? lane : 0)];
      }
      const int p = __builtin_amdgcn_readfirstlane(R.x);
      const int us = __builtin_amdgcn_readfirstlane(R.y) - gp0;
      const int nu = __builtin_amdgcn_readfirstlane(R.z);
      const int u0 = __builtin_amdgcn_readfirstlane(R.w);
      const double l = sv[p - gp0] * rp;
      if (lane < nu) sv[tg - gp0] -= l * sv[us + lane];
      for (int tt = lane + 64; tt < nu; tt += 64) sv[upd_tgt[u0 + tt] - gp0] -= l * sv[us + tt];
      if (lane == 0) sv[p - gp0] = l;
    }
    lds_barrier();
  }
  for (int e = t; e < seg; e += blockDim.x) a[gp0 + e] = sv[e];
}

// Top rows, eliminations by pack columns (all final): independent rows.
__global__ void k_rf_top_ext(int t0, int n, const int32_t* __restrict__ lo_split, const int32_t* __restrict__ ptr,
                             const int32_t* __restrict__ col, const int32_t* __restrict__ diag,
                             const int64_t* __restrict__ upd_ptr, const int32_t* __restrict__ upd_tgt,
                             double* __restrict__ a, double* __restrict__ rdg, int maxrow,
                             int32_t* __restrict__ status, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ double lds[];
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  double* w = lds + (size_t)wave * maxrow;
  const int i = t0 + blockIdx.x * nwave + wave;
  if (i >= n) return;
  rf_row(i, lo_split[i], false, ptr, col, diag, upd_ptr, upd_tgt, a, rdg, w, 0.0, status);
}

__global__ void k_fill_dbl(int64_t n, double* __restrict__ p, double v,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// dense[off[e]] = a[pos[e]] (to_dense) or a[pos[e]] = dense[off[e]]
__global__ void k_dense_xfer(int n, const int32_t* __restrict__ pos, const int64_t* __restrict__ off,
                             double* __restrict__ a, double* __restrict__ dense, int to_dense,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  if (to_dense) dense[off[e]] = a[pos[e]];
  else a[pos[e]] = dense[off[e]];
}

// ---------------------------------------- partitioned triangular solves
// X is an [n x ld] row-major block; each workgroup owns TW columns.  The
// rows of one pack (or of the top part) live in LDS for the whole solve;
// levels are separated by workgroup barriers.  LOWER entries of row i are
// [ptr[i], diag[i]); upper entries (diag[i], ptr[i+1]).

// xs[b0 + r][c] -= sum_{j in [j0, j1)} M[b0 + r][j] xs[j][c] for the nb rows
// of one block: M staged through LDS in 64 x 32 tiles (coalesced rows,
// zero outside [j0, j1)), the next tile loaded into registers while the
// current one is used; each thread accumulates up to four (row, column)
// pairs over a fully unrolled 32-wide tile.  xs rows are clamped to s - 1
// where the tile is zero, so every LDS index stays inside xs.
__device__ __forceinline__ void top_block_update(const double* __restrict__ M, int s, int b0, int nb, int j0, int j1,
                                        double* xs, int tw, double (*mt)[33]) {
  const int t = threadIdx.x;
  const int npair = nb * tw;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int rk[4], ck[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = t + k * 256;
    rk[k] = e < npair ? e / tw : 0;
    ck[k] = e < npair ? e - rk[k] * tw : 0;
  }
  // tile element e = t + 256 m (m < 8): row e >> 5, column e & 31; loaded
  // with clamped addresses and masked at the LDS store, so the loads of the
  // next tile stay in flight while the current one is used
  double nxt[8];
  auto load = [&](int jt) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = t + 256 * m, r = e >> 5, j = e & 31;
      nxt[m] = M[(size_t)(b0 + min(r, nb - 1)) * s + min(jt + j, s - 1)];
    }
  };
  if (j0 < j1) load(j0);
  for (int jt = j0; jt < j1; jt += 32) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = t + 256 * m, r = e >> 5, j = e & 31;
      mt[r][j] = (r < nb && jt + j < j1) ? nxt[m] : 0.0;
    }
    lds_barrier();
    if (jt + 32 < j1) load(jt + 32);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (t + k * 256 < npair) {
        const int r = rk[k], c = ck[k];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int j = 0; j < 32; j += 4) {
          a0 += mt[r][j] * xs[min(jt + j, s - 1) * tw + c];
          a1 += mt[r][j + 1] * xs[min(jt + j + 1, s - 1) * tw + c];
          a2 += mt[r][j + 2] * xs[min(jt + j + 2, s - 1) * tw + c];
          a3 += mt[r][j + 3] * xs[min(jt + j + 3, s - 1) * tw + c];
        }
        acc[k] += (a0 + a1) + (a2 + a3);
      }
    }
    lds_barrier();
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (t + k * 256 < npair) xs[(b0 + rk[k]) * tw + ck[k]] -= acc[k];
  }
  lds_barrier();
}

// Right-hand side of the top rows: X[i, c] <- scale X[i, c] - sum_p f(p)
// X[col(p), c] over the lower entries of top row i in pack columns
// ([ptr[i], lo_split[i])).  Reads only pack rows, so in place.  One thread
// per (row, column), four partial sums.
__global__ void k_top_rhs(int t0, int n, const int32_t* __restrict__ lo_split, const int32_t* __restrict__ ptr,
                          const int32_t* __restrict__ col, const double* __restrict__ fval,
                          double* __restrict__ X, int ld, int ncols, double scale,
                          const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t0 + blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= n || c >= ncols) return;
  double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
  const int p1 = lo_split[i];
  int p = ptr[i];
  for (; p + 3 < p1; p += 4) {
    const int j0 = col[p], j1 = col[p + 1], j2 = col[p + 2], j3 = col[p + 3];
    q0 += fval[p] * X[(size_t)j0 * ld + c];
    q1 += fval[p + 1] * X[(size_t)j1 * ld + c];
    q2 += fval[p + 2] * X[(size_t)j2 * ld + c];
    q3 += fval[p + 3] * X[(size_t)j3 * ld + c];
  }
  for (; p < p1; ++p) q0 += fval[p] * X[(size_t)col[p] * ld + c];
  X[(size_t)i * ld + c] = scale * X[(size_t)i * ld + c] - ((q0 + q1) + (q2 + q3));
}

// Products of the pack rows with the solved top rows, before the backward
// pack solves: X[i, c] -= sum_p f(p) X[col(p), c] over the upper entries
// of pack row i in top columns ([up_split[i], ptr[i+1])).  Reads only top
// rows, so in place.  One thread per (row, column), four partial sums.

// sum_p fval[p] X[col[p]][c] over p in [p0, p1) for columns c0 + 64 m
// (m < CPT) of one lane, the row's entries read as scalars (p0, p1
// wave-uniform), eight per pass with their X loads in flight; the next
// pass's entries and loads are issued before this pass's products (always,
// clamped, so every pass issues the same loads), and entries past p1 are
// masked where they are used.  Partial sums by (p - p0) mod 4; with TAIL0
// the entries past the last full group of four go to the first sum
// instead.  Combined as (s0 + s1) + (s2 + s3).
template <int CPT, bool TAIL0>
__device__ __forceinline__ void row_gather(int p0, int p1, const int32_t* __restrict__ col,
                                           const double* __restrict__ fval, const double* __restrict__ X, int ld,
                                           int c0, int ncols, double (&r)[CPT]) {
  double a[CPT][4];
#pragma unroll
  for (int k = 0; k < CPT; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) a[k][m] = 0.0;
  if (p1 <= p0) {
#pragma unroll
    for (int k = 0; k < CPT; ++k) r[k] = 0.0;
    return;
  }
  const int pfull = p0 + ((p1 - p0) & ~3);
  auto fetch = [&](int pb, double (&vv)[8], double (&xv)[8][CPT]) {
    int jj[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int pc = min(pb + m, p1 - 1);
      jj[m] = col[pc];
      vv[m] = fval[pc];
    }
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
      for (int k = 0; k < CPT; ++k) xv[m][k] = X[(size_t)jj[m] * ld + min(c0 + 64 * k, ncols - 1)];
  };
  double vv[8], xv[8][CPT];
  fetch(p0, vv, xv);
  for (int pb = p0; pb < p1; pb += 8) {
    double vn[8], xn[8][CPT];
    fetch(pb + 8 < p1 ? pb + 8 : pb, vn, xn);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int q = (TAIL0 && pb + m >= pfull) ? 0 : (m & 3);
      const double v = pb + m < p1 ? vv[m] : 0.0;
#pragma unroll
      for (int k = 0; k < CPT; ++k) a[k][q] += v * xv[m][k];
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      vv[m] = vn[m];
#pragma unroll
      for (int k = 0; k < CPT; ++k) xv[m][k] = xn[m][k];
    }
  }
#pragma unroll
  for (int k = 0; k < CPT; ++k) r[k] = (a[k][0] + a[k][1]) + (a[k][2] + a[k][3]);
}

// Batched forms (a wavefront per row, lane l taking columns c0 + l + 64 m):
// top rows X[i] = scale X[i] - (pack part of row i) X, and pack rows (only
// those with entries in top columns, listed in rows) X[i] -= (top part of
// row i) X.  The top rows sum in the same order as k_top_rhs, which
// serves single columns.
template <int CPT>
__global__ void __launch_bounds__(256) k_top_rhs_w(int t0, int n, const int32_t* __restrict__ lo_split,
                                                   const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                   const double* __restrict__ fval, double* __restrict__ X, int ld,
                                                   int ncols, double scale, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = t0 + __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (int)(threadIdx.x >> 6));
  if (i >= n) return;
  const int c0 = blockIdx.x * 64 * CPT + (threadIdx.x & 63);
  double r[CPT];
  row_gather<CPT, true>(ptr[i], lo_split[i], col, fval, X, ld, c0, ncols, r);
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = c0 + 64 * k;
    if (c < ncols) X[(size_t)i * ld + c] = scale * X[(size_t)i * ld + c] - r[k];
  }
}

template <int CPT>
__global__ void __launch_bounds__(256) k_pack_topmul_w(int nrows, const int32_t* __restrict__ rows,
                                                       const int32_t* __restrict__ up_split,
                                                       const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                       const double* __restrict__ fval, double* __restrict__ X,
                                                       int ld, int ncols, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int idx = __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (int)(threadIdx.x >> 6));
  if (idx >= nrows) return;
  const int i = rows[idx];
  const int c0 = blockIdx.x * 64 * CPT + (threadIdx.x & 63);
  double r[CPT];
  row_gather<CPT, false>(up_split[i], ptr[i + 1], col, fval, X, ld, c0, ncols, r);
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = c0 + 64 * k;
    if (c < ncols) X[(size_t)i * ld + c] -= r[k];
  }
}

// Rows of the inverse of one triangular CB x CB block, in solve order
// (LOWER: top down, terms j < i; upper: bottom up, terms j > i).  Thread
// (column c, segment seg) holds z[4 m + seg][c] in zr[m] and sums the terms
// j = 4 m + seg; the four segments of a column are adjacent lanes and
// combine their partial sums by DPP.  T is the strict triangle (zero
// elsewhere), so terms outside it, and entries of zr not yet solved (zero),
// add nothing; loops start or stop at the first term a row can need.
template <bool LOWER>
__device__ __forceinline__ void tri_inv_rows(const double (*T)[CB + 1], const double* rd, int c, int seg, int nb,
                                             double* zr) {
#pragma unroll
  for (int k = 0; k < CB; ++k) {
    const int i = LOWER ? k : CB - 1 - k;
    double a0 = (i == c && seg == 0) ? 1.0 : 0.0, a1 = 0.0;
    constexpr int M = CB / 4;
#pragma unroll
    for (int m = LOWER ? 0 : i / 4; m < (LOWER ? (i + 3) / 4 : M); ++m) {
      if (m & 1) a1 -= T[i][4 * m + seg] * zr[m];
      else a0 -= T[i][4 * m + seg] * zr[m];
    }
    double v = group_sum(a0 + a1, 4) * rd[i];
    v = (i < nb && c < nb) ? v : 0.0;
    zr[i >> 2] = seg == (i & 3) ? v : zr[i >> 2];
  }
}

// Inverses of the CB x CB diagonal blocks of a dense factor M (s x s,
// row-major, lower part L, upper part U): blockIdx.y = 0 inverts the lower
// triangle of block blockIdx.x (unit diagonal if lower_unit), 1 the upper
// triangle (unit if upper_unit).  Output dinv[(kb * 2 + part) * CB * CB],
// row-major CB x CB, zero outside the block's nb x nb corner.  With dinvT,
// also the inverse blocks of M^T (lower part U^T, upper part L^T), as the
// transposes.  256 threads: four lanes per column of the inverse
// (tri_inv_rows).
__global__ void __launch_bounds__(256) k_top_diag_inv(int s, const double* __restrict__ M, double* __restrict__ dinv,
                                                      int lower_unit, int upper_unit, double* __restrict__ dinvT,
                                                      const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double T[CB][CB + 1];   // strict triangle of the part, zero elsewhere
  __shared__ double rd[CB];          // 1 / diagonal (1 for a unit diagonal)
  const int kb = blockIdx.x, part = blockIdx.y;
  const int b0 = kb * CB, nb = min(CB, s - b0);
  const int t = threadIdx.x;
  const bool unit = part == 0 ? lower_unit != 0 : upper_unit != 0;
  {
    // all loads first (clamped into the block), then the stores
    double v[CB * CB / 256];
#pragma unroll
    for (int m = 0; m < CB * CB / 256; ++m) {
      const int e = t + 256 * m, r = e >> 6, cc = e & 63;
      v[m] = M[(size_t)(b0 + min(r, nb - 1)) * s + b0 + min(cc, nb - 1)];
    }
#pragma unroll
    for (int m = 0; m < CB * CB / 256; ++m) {
      const int e = t + 256 * m, r = e >> 6, cc = e & 63;
      const bool in = r < nb && cc < nb && (part == 0 ? cc < r : cc > r);
      T[r][cc] = in ? v[m] : 0.0;
    }
  }
  if (t < CB) rd[t] = (unit || t >= nb) ? 1.0 : 1.0 / M[(size_t)(b0 + t) * s + b0 + t];
  __syncthreads();
  const int c = t >> 2, seg = t & 3;
  double zr[CB / 4];
#pragma unroll
  for (int m = 0; m < CB / 4; ++m) zr[m] = 0.0;
  if (part == 0) tri_inv_rows<true>(T, rd, c, seg, nb, zr);
  else tri_inv_rows<false>(T, rd, c, seg, nb, zr);
  double* out = dinv + (size_t)(kb * 2 + part) * CB * CB;
#pragma unroll
  for (int m = 0; m < CB / 4; ++m) out[(4 * m + seg) * CB + c] = zr[m];
  if (dinvT) {
    // the transposed factor's inverse blocks: its lower triangle is this
    // upper one transposed and vice versa, and (T^-1)^T = (T^T)^-1
    double* ot = dinvT + (size_t)(kb * 2 + 1 - part) * CB * CB;
#pragma unroll
    for (int m = 0; m < CB / 4; ++m) ot[c * CB + 4 * m + seg] = zr[m];
  }
}

// xs[b0 + r][c] <- sum_j D[r][j] xs[b0 + j][c] for the nb rows of one block
// (D: a CB x CB inverse diagonal block, zero outside its nb x nb corner,
// staged through LDS; the unrolled sum clamps xs rows to s - 1 where D is
// zero).
__device__ __forceinline__ void top_diag_apply(const double* __restrict__ D, int s, int b0, int nb, double* xs, int tw,
                                      double (*dt)[CB + 1]) {
  const int t = threadIdx.x;
  stage_tile<256>(dt, D, CB, CB, CB, 0.0);
  lds_barrier();
  const int npair = nb * tw;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = t + k * 256;
    if (e < npair) {
      const int r = e / tw, c = e - r * tw;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
      for (int j = 0; j < CB; j += 4) {
        a0 += dt[r][j] * xs[min(b0 + j, s - 1) * tw + c];
        a1 += dt[r][j + 1] * xs[min(b0 + j + 1, s - 1) * tw + c];
        a2 += dt[r][j + 2] * xs[min(b0 + j + 2, s - 1) * tw + c];
        a3 += dt[r][j + 3] * xs[min(b0 + j + 3, s - 1) * tw + c];
      }
      acc[k] = (a0 + a1) + (a2 + a3);
    }
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = t + k * 256;
    if (e < npair) {
      const int r = e / tw, c = e - r * tw;
      xs[(b0 + r) * tw + c] = acc[k];
    }
  }
  lds_barrier();
}

// Single right-hand side of the power flow and adjoint solves, top rows:
// X[i] = scale X[i] - sum_{p in [ptr[i], lo_split[i])} fval[p] X[col[p]],
// a wavefront per row with its lanes splitting the entries (DPP sum).
__global__ void __launch_bounds__(256) k_top_rhs1(int t0, int n, const int32_t* __restrict__ lo_split,
                                                  const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                  const double* __restrict__ fval, double* __restrict__ X, int ld,
                                                  double scale, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = t0 + __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (int)(threadIdx.x >> 6));
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  const int p0 = ptr[i], p1 = lo_split[i];
  double a0 = 0.0, a1 = 0.0;
  for (int p = p0 + lane; p < p1; p += 128) {
    a0 += fval[p] * X[(size_t)col[p] * ld];
    if (p + 64 < p1) a1 += fval[p + 64] * X[(size_t)col[p + 64] * ld];
  }
  const double sum = group_sum(a0 + a1, 64);
  if (lane == 0) X[(size_t)i * ld] = scale * X[(size_t)i * ld] - sum;
}

// Single right-hand side: the dense top solves x <- U^-1 L^-1 x (with M,
// dinv of J_x^T: x <- L^-T U^-T x) for the s = n - t0 top rows (after
// k_top_rhs1), with the factor M (s x s, row-major) and the inverses of its
// diagonal blocks, in one workgroup of 1024 threads with x in LDS.  Per block of CB rows (forward, then backward): lane i is row i
// of the block and wavefront w takes 16 columns of each 256 of the solved
// part, so every product is a lane's own sum; the sixteen waves' partial
// sums are added by wave 0 through LDS, and the block's inverse is applied
// the same way (wave w its four columns), with no cross-lane reductions.
__global__ void __launch_bounds__(1024) k_top_solve1(int t0, int n, const double* __restrict__ M,
                                                     const double* __restrict__ dinv, double* __restrict__ X, int ld,
                                                     const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ double xs[];  // [s]
  __shared__ double part[16][CB + 1];
  __shared__ double rv[CB];
  const int s = n - t0;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int e = t; e < s; e += blockDim.x) xs[e] = X[(size_t)(t0 + e) * ld];
  const int nblk = (s + CB - 1) / CB;
  constexpr int CH = 16;   // columns per wave and pass
  lds_barrier();
  for (int q = 0; q < 2 * nblk; ++q) {
    const int bwd = q >= nblk ? 1 : 0;
    const int kb = bwd == 0 ? q : 2 * nblk - 1 - q;
    const int b0 = kb * CB, nb = min(CB, s - b0);
    // solved columns: forward [0, b0), backward [b0 + nb, s)
    const int j0 = bwd == 0 ? 0 : b0 + nb, j1 = bwd == 0 ? b0 : s;
    const double* D = dinv + (size_t)(kb * 2 + bwd) * CB * CB;
    const double* Mr = M + (size_t)(b0 + min(lane, nb - 1)) * s;
    double dv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) dv[c] = D[lane * CB + 4 * w + c];
    double a = 0.0;
    for (int jb = j0 + CH * w; jb < j1; jb += CH * 16) {
      double mv[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) mv[c] = Mr[min(jb + c, s - 1)];
#pragma unroll
      for (int c = 0; c < CH; ++c) a += (jb + c < j1 ? mv[c] : 0.0) * xs[min(jb + c, s - 1)];
    }
    part[w][lane] = a;
    lds_barrier();
    if (w == 0) {
      double sum = 0.0;
#pragma unroll
      for (int v = 0; v < 16; ++v) sum += part[v][lane];
      rv[lane] = lane < nb ? xs[min(b0 + lane, s - 1)] - sum : 0.0;
    }
    lds_barrier();
    double y = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) y += dv[c] * rv[4 * w + c];
    part[w][lane] = y;
    lds_barrier();
    if (w == 0) {
      double sum = 0.0;
#pragma unroll
      for (int v = 0; v < 16; ++v) sum += part[v][lane];
      if (lane < nb) xs[b0 + lane] = sum;
    }
    lds_barrier();
  }
  for (int e = t; e < s; e += blockDim.x) X[(size_t)(t0 + e) * ld] = xs[e];
}

// Dense forward and backward solves of the top rows (after k_top_rhs) with
// the factor M (s x s, row-major) and its inverse diagonal blocks dinv:
// per block of CB rows, subtract the products with the solved blocks
// (top_block_update), then multiply by the block's inverse.  The tw columns
// of one workgroup stay in LDS.  256 threads, tw <= 16.
__global__ void __launch_bounds__(256) k_top_dense(int t0, int n, const double* __restrict__ M,
                                                   const double* __restrict__ dinv, double* __restrict__ X,
                                                   int ld, int ncols, int tw, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ double xs[];
  __shared__ double mt[CB][33];
  __shared__ double dt[CB][CB + 1];
  const int s = n - t0;
  const int c0 = blockIdx.x * tw;
  const int t = threadIdx.x;
  for (int e = t; e < s * tw; e += blockDim.x) {
    const int r = e / tw, c = e - r * tw;
    xs[e] = (c0 + c < ncols) ? X[(size_t)(t0 + r) * ld + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int b0 = 0, kb = 0; b0 < s; b0 += CB, ++kb) {
    const int nb = min(CB, s - b0);
    top_block_update(M, s, b0, nb, 0, b0, xs, tw, mt);
    top_diag_apply(dinv + (size_t)(kb * 2) * CB * CB, s, b0, nb, xs, tw, dt);
  }
  const int nblk = (s + CB - 1) / CB;
  for (int kb = nblk - 1; kb >= 0; --kb) {
    const int b0 = kb * CB, nb = min(CB, s - b0);
    top_block_update(M, s, b0, nb, b0 + nb, s, xs, tw, mt);
    top_diag_apply(dinv + (size_t)(kb * 2 + 1) * CB * CB, s, b0, nb, xs, tw, dt);
  }
  for (int e = t; e < s * tw; e += blockDim.x) {
    const int r = e / tw, c = e - r * tw;
    if (c0 + c < ncols) X[(size_t)(t0 + r) * ld + c0 + c] = xs[e];
  }
}

// Staged pack solves: the pack's level lists, local columns, factor values
// and diagonal are copied to LDS first, so the level loop reads only LDS.
// For one right-hand side k_pack_solve_1 (below) is used when its level
// records fit in LDS; this kernel serves the packs where they do not.
// LDS layout: xs[nr*TW] | val[ne] | dg[nr] | rp[nr+1] (int) | lev[nlev+1]
// (int) | rows[nr] (short) | col[ne] (short).
__host__ __device__ __forceinline__ size_t pack_lds_bytes(int nr, int ne, int nlev, int tw) {
  size_t b = (size_t)nr * tw * 8 + (size_t)ne * 8 + (size_t)nr * 8 + (size_t)(nr + 1) * 4 +
             (size_t)(nlev + 1) * 4 + (size_t)nr * 2 + (size_t)ne * 2;
  return (b + 15) & ~(size_t)15;
}

// X_top <- S^-1 X_top (or S^-T X_top) with the dense inverse of the top
// block S computed once per point: out[r][c] = sum_k A[k * s + r]
// X[t0 + k][c], A k-major (S^-T for the J_x solves, S^-1 for J_x^T).  One
// workgroup per TW columns, staged in LDS; a thread per row, summing over
// k in order into two partial sums (even and odd k), so every element is
// the same whatever the batch width or split.  Sixteen rows of A in flight
// per pass.  blockDim a multiple of 64; rows past it loop.
template <int TW>
__global__ void __launch_bounds__(1024) k_top_inv_apply(int t0, int s, const double* __restrict__ A,
                                                         double* __restrict__ X, int ld, int ncols,
                                                         const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ double xs[];  // [s][TW]
  const int c0 = blockIdx.x * TW;
  for (int e = threadIdx.x; e < s * TW; e += blockDim.x) {
    const int k = e / TW, c = e - k * TW;
    xs[e] = c0 + c < ncols ? X[(size_t)(t0 + k) * ld + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int rb = 0; rb < s; rb += blockDim.x) {
    const int r = rb + threadIdx.x;
    const int rr = min(r, s - 1);
    double a0[TW], a1[TW];
#pragma unroll
    for (int c = 0; c < TW; ++c) a0[c] = a1[c] = 0.0;
    int k = 0;
    for (; k + 16 <= s; k += 16) {
      double av[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) av[m] = A[(size_t)(k + m) * s + rr];
#pragma unroll
      for (int m = 0; m < 16; m += 2)
#pragma unroll
        for (int c = 0; c < TW; ++c) {
          a0[c] += av[m] * xs[(k + m) * TW + c];
          a1[c] += av[m + 1] * xs[(k + m + 1) * TW + c];
        }
    }
    for (; k < s; ++k) {
      const double av = A[(size_t)k * s + rr];
#pragma unroll
      for (int c = 0; c < TW; ++c) {
        if (k & 1) a1[c] += av * xs[k * TW + c];
        else a0[c] += av * xs[k * TW + c];
      }
    }
    if (r < s) {
#pragma unroll
      for (int c = 0; c < TW; ++c)
        if (c0 + c < ncols) X[(size_t)(t0 + r) * ld + c0 + c] = a0[c] + a1[c];
    }
  }
}

template <int TW, bool FWD, bool UNIT>
__global__ void __launch_bounds__(256) k_pack_solve_s(const int32_t* __restrict__ pack_ptr, const int32_t* __restrict__ lev,
                               const int32_t* __restrict__ lev_off, const int32_t* __restrict__ lrows,
                               const int32_t* __restrict__ rp, const int32_t* __restrict__ epos,
                               const int16_t* __restrict__ ecol, const int32_t* __restrict__ diag,
                               const int32_t* __restrict__ up_split, const int32_t* __restrict__ ptr,
                               const int32_t* __restrict__ col, const double* __restrict__ val,
                               double* __restrict__ X, int ld, int ncols, double scale,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ double smem[];
  const int q = blockIdx.x;
  const int c0 = blockIdx.y * TW;
  const int r0 = pack_ptr[q], nr = pack_ptr[q + 1] - r0;
  const int e0 = rp[r0], ne = rp[r0 + nr] - e0;
  const int l0 = lev_off[q], nlev = lev_off[q + 1] - l0;
  const int base_row = lev[l0];
  double* xs = smem;
  double* sv = xs + (size_t)nr * TW;
  double* dg = sv + ne;
  int* srp = (int*)(dg + nr);
  int* slev = srp + nr + 1;
  short* srow = (short*)(slev + nlev + 1);
  short* scol = srow + nr;
  const int t = threadIdx.x;
  const int bd = blockDim.x;
  // staging: each pass issues all of a thread's loads (16 entries, or 4
  // rows) before its stores, with addresses clamped into range
  for (int eb = t; eb < ne; eb += 16 * bd) {
    int ps[16];
    int16_t cs[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int e = min(eb + m * bd, ne - 1);
      ps[m] = epos[e0 + e];
      cs[m] = ecol[e0 + e];
    }
    double vs[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) vs[m] = val[ps[m]];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int e = eb + m * bd;
      if (e < ne) {
        sv[e] = vs[m];
        scol[e] = cs[m];
      }
    }
  }
  for (int rb = t; rb <= nr; rb += 4 * bd) {
    int v[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = rp[r0 + min(rb + m * bd, nr)];
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (rb + m * bd <= nr) srp[rb + m * bd] = v[m] - e0;
  }
  for (int rb = t; rb < nr; rb += 4 * bd) {
    int di[4], lr[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = min(rb + m * bd, nr - 1);
      di[m] = UNIT ? 0 : diag[r0 + r];
      lr[m] = lrows[base_row + r];
    }
    double dv[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) dv[m] = UNIT ? 1.0 : val[di[m]];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = rb + m * bd;
      if (r < nr) {
        if (!UNIT) dg[r] = dv[m];
        srow[r] = (short)(lr[m] - r0);
      }
    }
  }
  for (int k = t; k <= nlev; k += bd) slev[k] = lev[l0 + k] - base_row;
  for (int eb = t; eb < nr * TW; eb += 4 * bd) {
    double xv[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int ec = min(eb + m * bd, nr * TW - 1);
      const int r = ec / TW, c = ec - r * TW;
      const int i = r0 + r;
      double acc = 0.0;
      if (c0 + c < ncols) {
        if (FWD) {
          acc = scale * X[(size_t)i * ld + c0 + c];
        } else {
          // solved top rows: independent products, two partial sums
          double a0 = 0.0, a1 = 0.0;
          const int p1 = ptr[i + 1];
          int p = up_split[i];
          for (; p + 1 < p1; p += 2) {
            a0 += val[p] * X[(size_t)col[p] * ld + c0 + c];
            a1 += val[p + 1] * X[(size_t)col[p + 1] * ld + c0 + c];
          }
          if (p < p1) a0 += val[p] * X[(size_t)col[p] * ld + c0 + c];
          acc = X[(size_t)i * ld + c0 + c] - (a0 + a1);
        }
      }
      xv[m] = acc;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (eb + m * bd < nr * TW) xs[eb + m * bd] = xv[m];
  }
  __syncthreads();
  // Level loop.  A level of nrow rows has nrow * TW (row, column) pairs; when
  // that is below the block size, G = 2^lg lanes share one pair, each
  // summing every G-th entry of the row (four partial sums, so the LDS loads
  // of a row overlap), and the G partial sums are combined by butterfly
  // shuffles inside the wavefront (groups of G lanes are aligned).
  const int nthr = blockDim.x;
  for (int lv = 0; lv < nlev; ++lv) {
    const int a = slev[lv], nrow = slev[lv + 1] - a;
    const int pairs = nrow * TW;
    int lg = 0;
    while (lg < 6 && (pairs << (lg + 1)) <= nthr) ++lg;
    const int G = 1 << lg;
    const int work = pairs << lg;
    for (int w0 = 0; w0 < work; w0 += nthr) {
      const int w = w0 + t;
      const bool act = w < work;
      const int pair = w >> lg, seg = w & (G - 1);
      const int rk = pair / TW;
      const int cc = pair - rk * TW;
      int r = 0;
      double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
      if (act) {
        r = srow[a + rk];
        const int e1 = srp[r + 1];
        int e = srp[r] + seg;
        for (; e + 3 * G < e1; e += 4 * G) {
          const int j0 = scol[e], j1 = scol[e + G], j2 = scol[e + 2 * G], j3 = scol[e + 3 * G];
          q0 += sv[e] * xs[j0 * TW + cc];
          q1 += sv[e + G] * xs[j1 * TW + cc];
          q2 += sv[e + 2 * G] * xs[j2 * TW + cc];
          q3 += sv[e + 3 * G] * xs[j3 * TW + cc];
        }
        for (; e < e1; e += G) q0 += sv[e] * xs[scol[e] * TW + cc];
      }
      double part = (q0 + q1) + (q2 + q3);
      part = group_sum(part, G);
      if (act && seg == 0) {
        double acc = xs[r * TW + cc] - part;
        if (!UNIT) acc /= dg[r];
        xs[r * TW + cc] = acc;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < nr * TW; e += blockDim.x) {
    const int r = e / TW, c = e - r * TW;
    if (c0 + c < ncols) X[(size_t)(r0 + r) * ld + c0 + c] = xs[e];
  }
}

// Single right-hand side pack solves (power flow Newton steps and the
// adjoint).  A level costs the instructions of one wavefront more than
// memory, so the loop is kept short: G = 2^lg lanes share a row, with lg
// per level from the host (enough lanes for two entries each on the
// level's longest row, at most 64, at most 256 lanes in all); each lane's
// two entries, the row's position, right-hand side and reciprocal pivot
// are loaded during the previous level (only the solved inputs xs[j]
// depend on earlier levels); entries past a row's end read a zero pad
// (value 0, column nr, xs[nr] = 0), so the sums need no masks; longer rows
// loop over the rest (only in levels the host marks), and levels of more
// than 256 / G rows take further passes without prefetch.  The loop is
// unrolled by two so the prefetched state alternates between two register
// sets.
// FWD: entries [ptr[i], diag[i]), x_i = scale b_i - sum; backward: entries
// (diag[i], up_split[i]), x_i = b_i - sum(top columns) - sum; UNIT = false
// multiplies by the staged 1 / u_ii.
// LDS: xs[nr + 1] | val[ne + 1] | 1/dg[nr] | unit[nr] (int2: row | length
// << 16, first entry) | rp[nr + 1] (int) | lev[nlev + 1] (int: first
// position | lg << 16 | long rows << 19) | rows[nr] (short) | col[ne + 1]
// (short).
__host__ __device__ __forceinline__ size_t pack1_lds_bytes(int nr, int ne, int nlev) {
  size_t b = (size_t)(nr + 1) * 8 + (size_t)(ne + 1) * 8 + (size_t)nr * 8 + (size_t)nr * 8 + (size_t)(nr + 1) * 4 +
             (size_t)(nlev + 1) * 4 + (size_t)nr * 2 + (size_t)(ne + 1) * 2;
  return (b + 15) & ~(size_t)15;
}

template <bool FWD, bool UNIT>
__global__ void __launch_bounds__(256) k_pack_solve_1(const int32_t* __restrict__ pack_ptr, const int32_t* __restrict__ lev,
                               const int32_t* __restrict__ lev_off, const int8_t* __restrict__ lev_lg,
                               const int32_t* __restrict__ lrows,
                               const int32_t* __restrict__ rp, const int32_t* __restrict__ epos,
                               const int16_t* __restrict__ ecol, const int32_t* __restrict__ diag,
                               const int32_t* __restrict__ up_split, const int32_t* __restrict__ ptr,
                               const int32_t* __restrict__ col, const double* __restrict__ val,
                               double* __restrict__ X, int ld, double scale, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ double smem[];
  const int q = blockIdx.x;
  const int r0 = pack_ptr[q], nr = pack_ptr[q + 1] - r0;
  const int e0 = rp[r0], ne = rp[r0 + nr] - e0;
  const int l0 = lev_off[q], nlev = lev_off[q + 1] - l0;
  const int base_row = lev[l0];
  double* xs = smem;
  double* sv = xs + nr + 1;
  double* rdg = sv + ne + 1;
  int2* sun = reinterpret_cast<int2*>(rdg + nr);
  int* srp = reinterpret_cast<int*>(sun + nr);
  int* slev = srp + nr + 1;
  short* srow = reinterpret_cast<short*>(slev + nlev + 1);
  short* scol = srow + nr;
  const int t = threadIdx.x;
  const int bd = blockDim.x;
  // Staging.  The first pass of the entries and of every per-row and
  // per-level array is loaded at once, then what depends on it (factor
  // values, pivots, the first two top-column terms of backward rows and
  // their solved values), and only then stored to LDS; further passes
  // (packs of more than 8192 entries or 1024 rows) and longer top-column
  // products follow.  Indices are clamped into their arrays; a pack
  // without entries reads entry 0 of the LU values.
  constexpr int EP = 32, RP = 4;
  {
    const bool has_e = ne > 0;
    int ps[EP];
    int16_t cs[EP];
#pragma unroll
    for (int m = 0; m < EP; ++m) {
      const int gi = has_e ? e0 + min(t + m * bd, ne - 1) : 0;
      ps[m] = epos[gi];
      cs[m] = ecol[gi];
    }
    int rpv[RP + 1];
#pragma unroll
    for (int m = 0; m <= RP; ++m) rpv[m] = rp[r0 + min(t + m * bd, nr)];
    int di[RP], lr[RP], ri[RP];
#pragma unroll
    for (int m = 0; m < RP; ++m) {
      ri[m] = r0 + min(t + m * bd, nr - 1);
      di[m] = UNIT ? 0 : diag[ri[m]];
      lr[m] = lrows[base_row + min(t + m * bd, nr - 1)];
    }
    const int kl = min(t, nlev);
    const int lvw = lev[l0 + kl];
    const int lgw = t < nlev ? (int)lev_lg[l0 + t] : 0;
    double xi[RP];
    int us[RP], pe[RP];
#pragma unroll
    for (int m = 0; m < RP; ++m) {
      xi[m] = X[(size_t)ri[m] * ld];
      us[m] = FWD ? 0 : up_split[ri[m]];
      pe[m] = FWD ? 0 : ptr[ri[m] + 1];
    }
    double vs[EP];
#pragma unroll
    for (int m = 0; m < EP; ++m) vs[m] = val[has_e ? ps[m] : 0];
    double dv[RP];
#pragma unroll
    for (int m = 0; m < RP; ++m) dv[m] = UNIT ? 1.0 : val[di[m]];
    // backward: the first two terms of each row's solved top-column product
    int tc[RP][2];
    double tv[RP][2];
    if (!FWD) {
#pragma unroll
      for (int m = 0; m < RP; ++m)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int pp = min(us[m] + k, pe[m] - 1);
          tc[m][k] = col[pp];
          tv[m][k] = val[pp];
        }
    }
    double tx[RP][2];
    if (!FWD) {
#pragma unroll
      for (int m = 0; m < RP; ++m)
#pragma unroll
        for (int k = 0; k < 2; ++k) tx[m][k] = X[(size_t)tc[m][k] * ld];
    }
#pragma unroll
    for (int m = 0; m < EP; ++m) {
      const int e = t + m * bd;
      if (e < ne) {
        sv[e] = vs[m];
        scol[e] = cs[m];
      }
    }
#pragma unroll
    for (int m = 0; m <= RP; ++m)
      if (t + m * bd <= nr) srp[t + m * bd] = rpv[m] - e0;
    if (t <= nlev) slev[t] = (lvw - base_row) | (lgw << 16);
#pragma unroll
    for (int m = 0; m < RP; ++m) {
      const int r = t + m * bd;
      double acc;
      if (FWD) {
        acc = scale * xi[m];
      } else {
        // independent products, two partial sums
        const int p1 = pe[m];
        double a0 = us[m] < p1 ? tv[m][0] * tx[m][0] : 0.0;
        double a1 = us[m] + 1 < p1 ? tv[m][1] * tx[m][1] : 0.0;
        int p = us[m] + 2;
        for (; p + 1 < p1; p += 2) {
          a0 += val[p] * X[(size_t)col[p] * ld];
          a1 += val[p + 1] * X[(size_t)col[p + 1] * ld];
        }
        if (p < p1) a0 += val[p] * X[(size_t)col[p] * ld];
        acc = xi[m] - (a0 + a1);
      }
      if (r < nr) {
        if (!UNIT) rdg[r] = 1.0 / dv[m];
        srow[r] = (short)(lr[m] - r0);
        xs[r] = acc;
      }
    }
  }
  if (t == 0) {
    sv[ne] = 0.0;
    scol[ne] = (short)nr;
    xs[nr] = 0.0;
  }
  // further passes
  for (int eb = t + EP * bd; eb < ne; eb += EP * bd) {
    int ps[EP];
    int16_t cs[EP];
#pragma unroll
    for (int m = 0; m < EP; ++m) {
      const int e = min(eb + m * bd, ne - 1);
      ps[m] = epos[e0 + e];
      cs[m] = ecol[e0 + e];
    }
    double vs[EP];
#pragma unroll
    for (int m = 0; m < EP; ++m) vs[m] = val[ps[m]];
#pragma unroll
    for (int m = 0; m < EP; ++m) {
      const int e = eb + m * bd;
      if (e < ne) {
        sv[e] = vs[m];
        scol[e] = cs[m];
      }
    }
  }
  for (int k = t + (RP + 1) * bd; k <= nr; k += bd) srp[k] = rp[r0 + k] - e0;
  for (int k = t + bd; k <= nlev; k += bd) slev[k] = (lev[l0 + k] - base_row) | ((k < nlev ? (int)lev_lg[l0 + k] : 0) << 16);
  for (int r = t + RP * bd; r < nr; r += bd) {
    const int i = r0 + r;
    double acc;
    if (FWD) {
      acc = scale * X[(size_t)i * ld];
    } else {
      double a0 = 0.0, a1 = 0.0;
      const int p1 = ptr[i + 1];
      int p = up_split[i];
      for (; p + 1 < p1; p += 2) {
        a0 += val[p] * X[(size_t)col[p] * ld];
        a1 += val[p + 1] * X[(size_t)col[p + 1] * ld];
      }
      if (p < p1) a0 += val[p] * X[(size_t)col[p] * ld];
      acc = X[(size_t)i * ld] - (a0 + a1);
    }
    if (!UNIT) rdg[r] = 1.0 / val[diag[i]];
    srow[r] = (short)(lrows[base_row + r] - r0);
    xs[r] = acc;
  }
  __syncthreads();
  // one record per level position: the row, its entry count and first entry
  for (int k = t; k < nr; k += bd) {
    const int r = srow[k];
    const int b = srp[r];
    sun[k] = make_int2(r | ((srp[r + 1] - b) << 16), b);
  }
  __syncthreads();
  if (nlev == 0) return;
  // a lane's unit at a level: its row, first entry, row end, first two
  // (column, value) pairs, right-hand side and reciprocal pivot
  struct Unit {
    int r, e, e1;
    int j[2];
    double v[2];
    double xr, rd;
  };
  auto fetch = [&](const int2 rec, int seg, int G, Unit& u) {
    u.r = rec.x & 0xFFFF;
    u.e = rec.y + seg;
    u.e1 = rec.y + (rec.x >> 16);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int em = u.e + m * G;
      const int ec = em < u.e1 ? em : ne;
      u.j[m] = scol[ec];
      u.v[m] = sv[ec];
    }
    u.xr = xs[u.r];
    u.rd = UNIT ? 1.0 : rdg[u.r];
  };
  // the unit of the level whose words are wa (first position | lg << 16)
  // and wb (the next level's)
  auto fetch_level = [&](int wa, int wb, Unit& u) {
    const int a = wa & 0xFFFF, nrow = (wb & 0xFFFF) - a, lg = (wa >> 16) & 7;
    fetch(sun[max(a + min(t >> lg, nrow - 1), 0)], t & ((1 << lg) - 1), 1 << lg, u);
  };
  // the unit's sum over its lanes and the row's new value
  auto finish = [&](const Unit& u, const double (&x)[2], int lg, bool longrows, int seg, bool act) {
    const int G = 1 << lg;
    double part = fma(u.v[1], x[1], u.v[0] * x[0]);
    if (longrows && act)
      for (int e = u.e + 2 * G; e < u.e1; e += G) part += sv[e] * xs[scol[e]];
    part = group_sum(part, G);
    if (act && seg == 0) {
      double acc = u.xr - part;
      if (!UNIT) acc *= u.rd;
      xs[u.r] = acc;
    }
  };
  int w0 = slev[0], w1 = slev[1], w2 = slev[min(2, nlev)];
  Unit ua, ub;
  fetch_level(w0, w1, ua);
  auto step = [&](int lv, const Unit& cur, Unit& nxt) {
    const int a = w0 & 0xFFFF, nrow = (w1 & 0xFFFF) - a, lg = (w0 >> 16) & 7;
    const bool longrows = (w0 >> 19) & 1;
    const int G = 1 << lg, work = nrow << lg, seg = t & (G - 1);
    double x[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) x[m] = xs[cur.j[m]];
    // keep these loads ahead of the next level's (the scheduler would issue
    // the longer chain first and put its round trip before the sums)
    __builtin_amdgcn_sched_barrier(0);
    // the next level's unit (after the last level the indices stay in range
    // and the values go unused) and the word of the level after it
    const int w3 = slev[min(lv + 3, nlev)];
    fetch_level(w1, w2, nxt);
    finish(cur, x, lg, longrows, seg, t < work);
    // levels wider than one pass of the workgroup
    for (int w = t + bd; w - t < work; w += bd) {
      Unit u;
      fetch(sun[a + min(w >> lg, nrow - 1)], seg, G, u);
      double xu[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) xu[m] = xs[u.j[m]];
      finish(u, xu, lg, longrows, seg, w < work);
    }
    __syncthreads();
    w0 = w1;
    w1 = w2;
    w2 = w3;
  };
  for (int lv = 0; lv < nlev; lv += 2) {
    step(lv, ua, ub);
    if (lv + 1 < nlev) step(lv + 1, ub, ua);
  }
  for (int r = t; r < nr; r += bd) X[(size_t)(r0 + r) * ld] = xs[r];
}

// Batched pack solves in place in global memory, for many right-hand
// sides.  One workgroup (16 wavefronts) per (pack, 64-column tile); the
// pack's column indices and row ranges are staged in LDS, factor values
// and X are read from global memory (the rows a pack reads are written by
// the same workgroup before a workgroup barrier, or are final top rows).
// Per level, a wavefront takes one unit = (row, chunk of 64 / G columns)
// with G lanes per column summing every G-th entry (G = 2^lg chosen so
// the level's units fill the wavefronts), butterfly-reduced.
// FWD: entries [ptr[i], diag[i]) (L, or U^T), x_i = scale b_i - sum;
// backward: entries (diag[i], ptr[i+1]) (U, or L^T, top columns included),
// x_i = b_i - sum; UNIT = false multiplies by 1 / val[diag[i]].
// LDS: scol[seg] | sptr[nr + 1] | sdiag[nr] | srow[nr] | slev[nlev + 1] |
// srd[nr] (double), seg = nnz of the pack's CSR rows.
__host__ __device__ __forceinline__ size_t packg_lds_bytes(int nr, int seg, int nlev) {
  size_t b = (size_t)seg * 4 + (size_t)(nr + 1) * 4 + (size_t)nr * 8 + (size_t)(nlev + 1) * 4;
  b = (b + 7) & ~(size_t)7;
  return b + (size_t)nr * 8;
}

template <bool FWD, bool UNIT>
__global__ void __launch_bounds__(1024) k_pack_solve_g(const int32_t* __restrict__ pack_ptr,
                                                       const int32_t* __restrict__ lev,
                                                       const int32_t* __restrict__ lev_off,
                                                       const int32_t* __restrict__ lrows,
                                                       const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ diag,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val, double* __restrict__ X,
                                                       int ld, int ncols, double scale,
                                                       const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ int32_t smi[];
  const int q = blockIdx.x;
  const int c0 = blockIdx.y * 64;
  const int r0 = pack_ptr[q], nr = pack_ptr[q + 1] - r0;
  const int l0 = lev_off[q], nlev = lev_off[q + 1] - l0;
  const int gp0 = ptr[r0], seg = ptr[r0 + nr] - gp0;
  const int base_row = lev[l0];
  int32_t* scol = smi;
  int32_t* sptr = scol + seg;
  int32_t* sdiag = sptr + nr + 1;
  int32_t* srow = sdiag + nr;
  int32_t* slev = srow + nr;
  size_t off = (size_t)seg + (nr + 1) + 2 * (size_t)nr + (nlev + 1);
  off = (off + 1) & ~(size_t)1;
  double* srd = (double*)(smi + off);
  const int t = threadIdx.x;
  stage_1d(scol, col + gp0, seg);
  for (int r = t; r <= nr; r += blockDim.x) sptr[r] = ptr[r0 + r] - gp0;
  for (int r = t; r < nr; r += blockDim.x) {
    const int dg = diag[r0 + r];
    sdiag[r] = dg - gp0;
    srow[r] = lrows[base_row + r] - r0;
    srd[r] = UNIT ? 1.0 : 1.0 / val[dg];
  }
  for (int k = t; k <= nlev; k += blockDim.x) slev[k] = lev[l0 + k] - base_row;
  __syncthreads();
  const int wave = t >> 6, lane = t & 63, nwave = blockDim.x >> 6;
  for (int lv = 0; lv < nlev; ++lv) {
    const int a = slev[lv], nrow = slev[lv + 1] - a;
    int lg = 0;
    while (lg < 4 && (nrow << (lg + 1)) <= nwave) ++lg;
    const int G = 1 << lg;
    const int units = nrow << lg;
    const int segl = lane & (G - 1);
    for (int u = wave; u < units; u += nwave) {
      const int k = u >> lg, qch = u & (G - 1);
      // the unit's row is the same in every lane: keep its bounds scalar
      const int rl = __builtin_amdgcn_readfirstlane(srow[a + k]);
      const int i = r0 + rl;
      const int c = c0 + (qch << (6 - lg)) + (lane >> lg);
      const bool cok = c < ncols;
      const int cl = cok ? c : ncols - 1;   // in-bounds column for loads
      const int e0 = __builtin_amdgcn_readfirstlane(FWD ? sptr[rl] : sdiag[rl] + 1);
      const int e1 = __builtin_amdgcn_readfirstlane(FWD ? sdiag[rl] : sptr[rl + 1]);
      const size_t xi = (size_t)i * ld + cl;
      const double xown = X[xi];
      // entries in groups of 8 G: eight independent loads per lane in flight,
      // out-of-range slots read entry e0 with weight zero
      double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
      for (int eb = e0; eb < e1; eb += 8 * G) {
        double v[8], xv[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int e = eb + m * G + segl;
          const bool in = e < e1;
          const int ec = in ? e : e0;
          v[m] = in ? val[gp0 + ec] : 0.0;
          xv[m] = X[(size_t)scol[ec] * ld + cl];
        }
        q0 += v[0] * xv[0] + v[4] * xv[4];
        q1 += v[1] * xv[1] + v[5] * xv[5];
        q2 += v[2] * xv[2] + v[6] * xv[6];
        q3 += v[3] * xv[3] + v[7] * xv[7];
      }
      double part = (q0 + q1) + (q2 + q3);
      part = group_sum(part, G);
      if (cok && segl == 0) {
        double xnew = (FWD ? scale * xown : xown) - part;
        if (!UNIT) xnew *= srd[rl];
        X[xi] = xnew;
      }
    }
    __syncthreads();
  }
}

// Batched pack solves with the pack's right-hand-side tile in LDS: one
// workgroup of 1024 threads per (pack, TW-column tile).  Staged in LDS: the
// tile X[r0 .. r1) x [c0, c0 + TW) (forward: times scale; backward: the
// products with the top rows are already subtracted by k_pack_topmul_w), and
// the pack program of the
// direction: local columns (int16), rows in level order with each row's
// first entry and length in one word, level offsets.  Factor values come from pval, a copy in program order
// (one load per entry); 1 / u_ii from rdg (non-unit factors).  Per level a
// wavefront covers R rows x TW columns (lanes: column fastest, then G lanes
// sharing one row's entries, then R row slots; R G TW = 64); R shrinks on
// narrow levels so that more lanes share a row.  Eight entries per lane are
// in flight at a time.
// With SV the values are staged too and every level touches only LDS.
// LDS: [sval[ne] (double, SV)] | xs[nr TW] (double) | smeta[nr + 1] |
// slev[nlev + 1] (int) | srow[nr] | scol[ne] (int16).
__host__ __device__ __forceinline__ size_t packt_lds_bytes(int nr, int ne, int nlev, int tw, bool sv) {
  return (sv ? (size_t)ne * 8 : 0) + (size_t)nr * tw * 8 + (size_t)(nr + 1) * 4 + (size_t)(nlev + 1) * 4 +
         (size_t)nr * 2 + (size_t)ne * 2 + 2 * TAIL_MAX + 16;
}

// Dense tail of a pack (the rows T near the subtree roots, rows sT[0 .. nT)
// of the tile, ascending): x_T <- M x_T with M the dense inverse of the
// factor's T x T block (row-major, leading dimension TAIL_MAX; lower
// triangular for the forward solves, upper for the backward ones).  Thread
// t computes column t % TW of rows t / TW + k (1024 / TW), k < passes, all
// reads before the barrier, then the stores.
template <int TW>
__device__ __forceinline__ void tail_apply(double* xs, const int16_t* sT, int nT, const double* __restrict__ M,
                                           bool lower) {
  constexpr int RPP = 1024 / TW;
  constexpr int NP = (TAIL_MAX + RPP - 1) / RPP;
  const int t = threadIdx.x;
  const int c = t & (TW - 1), i0 = t / TW;
  double acc[NP];
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) {
    const int i = i0 + pp * RPP;
    double a0 = 0.0, a1 = 0.0;
    if (i < nT) {
      const double* mrow = M + (size_t)i * TAIL_MAX;
      const int k0 = lower ? 0 : i, k1 = lower ? i + 1 : nT;
      int k = k0;
      for (; k + 8 <= k1; k += 8) {
        double mv[8], xv[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          mv[m] = mrow[k + m];
          xv[m] = xs[sT[k + m] * TW + c];
        }
#pragma unroll
        for (int m = 0; m < 8; m += 2) {
          a0 += mv[m] * xv[m];
          a1 += mv[m + 1] * xv[m + 1];
        }
      }
      for (; k < k1; ++k) a0 += mrow[k] * xs[sT[k] * TW + c];
    }
    acc[pp] = a0 + a1;
  }
  lds_barrier();
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) {
    const int i = i0 + pp * RPP;
    if (i < nT) xs[sT[i] * TW + c] = acc[pp];
  }
  lds_barrier();
}

// tail_apply for 16 columns on the FP64 matrix cores: wave w < 8 forms rows
// 16 w .. 16 w + 15 of M x_T (v_mfma_f64_16x16x4f64: A = rows of M read
// straight from memory, lane i + 16 k holding M(i, k); B = the tail rows of
// the tile, lane c + 16 k holding x(k, c); the result's lane c + 16 q holds
// rows q + 4 r of column c), over the triangle's k range in chunks of 32,
// the next chunk's operands loaded during the current chunk's products.
// Entries of M outside the triangle or past nT are not used.
__device__ __forceinline__ void tail_apply_mfma(double* xs, const int16_t* sT, int nT, const double* __restrict__ M,
                                                bool lower) {
  constexpr int TW = 16;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int li = l & 15, lk = l >> 4;
  const int rb = w;
  const bool active = rb < 8 && 16 * rb < nT;
  dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
  if (active) {
    const int i = 16 * rb + li;
    const int ka = lower ? 0 : 16 * rb, kb = lower ? min(16 * rb + 16, nT) : nT;
    const double* mrow = M + (size_t)i * TAIL_MAX;
    double av[8], bv[8];
    auto load = [&](int k0) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int k = k0 + 4 * m + lk;
        const int kc = min(k, nT - 1);
        const bool inA = i < nT && k < kb && (lower ? k <= i : k >= i);
        const double g = mrow[kc];
        av[m] = inA ? g : 0.0;
        bv[m] = k < kb ? xs[sT[kc] * TW + li] : 0.0;
      }
    };
    load(ka);
    for (int k0 = ka; k0 < kb; k0 += 32) {
      double a2[8], b2[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        a2[m] = av[m];
        b2[m] = bv[m];
      }
      if (k0 + 32 < kb) load(k0 + 32);
#pragma unroll
      for (int m = 0; m < 8; ++m) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[m], b2[m], acc, 0, 0, 0);
    }
  }
  lds_barrier();
  if (active) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + lk + 4 * r;
      if (row < nT) xs[sT[row] * TW + li] = acc[r];
    }
  }
  lds_barrier();
}

template <int TW>
__device__ __forceinline__ void tail_apply_any(double* xs, const int16_t* sT, int nT, const double* __restrict__ M,
                                               bool lower) {
  if constexpr (TW == 16) tail_apply_mfma(xs, sT, nT, M, lower);
  else tail_apply<TW>(xs, sT, nT, M, lower);
}

// Optional fusions of the batched pack solves: forward, the right-hand side
// R = -J_u V staged from V (J_u in CSR over the state rows: jp, jc, jv; V
// [n_u x ncols] with leading dimension ldv) instead of read from X;
// backward, the top-column products of the pack rows listed in tmrows
// [tmoff[q] .. tmoff[q+1]) subtracted after staging (their values from val,
// the solved top rows from X).
struct PackFuse {
  const int32_t* jp = nullptr;
  const int32_t* jc = nullptr;
  const double* jv = nullptr;
  const double* V = nullptr;
  int ldv = 0;
  const int32_t* tmoff = nullptr;
  const int32_t* tmrows = nullptr;
};

template <int TW, bool FWD, bool UNIT, bool SV>
__global__ void __launch_bounds__(1024) k_pack_solve_t(const int32_t* __restrict__ pack_ptr,
                                                       const int32_t* __restrict__ lev,
                                                       const int32_t* __restrict__ lev_off,
                                                       const int32_t* __restrict__ lrows,
                                                       const int32_t* __restrict__ rp,
                                                       const int16_t* __restrict__ ecol,
                                                       const double* __restrict__ pval,
                                                       const double* __restrict__ rdg,
                                                       const int32_t* __restrict__ up_split,
                                                       const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val, double* __restrict__ X,
                                                       int ld, int ncols, double scale, int npacks, int ntiles,
                                                       const int32_t* __restrict__ toff,
                                                       const int16_t* __restrict__ trows,
                                                       const double* __restrict__ tinv,
                                                       const int32_t* __restrict__ skip, PackFuse fz) {
  if (skip && *skip) return;
  constexpr int S = 64 / TW;   // lanes per column in a wavefront
  constexpr int LGS = S == 8 ? 3 : S == 4 ? 2 : S == 2 ? 1 : 0;
  extern __shared__ double smem[];
  // XCD-aware mapping: workgroup b runs on XCD b % 8; pack q belongs to XCD
  // q % 8, whose workgroups take its packs' column tiles in order, so the
  // tiles of one pack share that XCD's L2 (factor values, columns)
  const int xcd = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int qq = jx / ntiles;
  const int q = xcd + 8 * qq;
  if (q >= npacks) return;
  const int c0 = (jx - qq * ntiles) * TW;
  const int r0 = pack_ptr[q], nr = pack_ptr[q + 1] - r0;
  const int e0 = rp[r0], ne = rp[r0 + nr] - e0;
  const int l0 = lev_off[q], nlev = lev_off[q + 1] - l0;
  const int base_row = lev[l0];
  const int nprog = lev[l0 + nlev] - base_row;   // rows of the program (the tail rows are not
                                                 // in the backward one)
  const int tq = toff ? toff[q] : 0, nT = toff ? toff[q + 1] - tq : 0;
  double* sval = smem;
  double* xs = smem + (SV ? ne : 0);
  int* smeta = (int*)(xs + (size_t)nr * TW);
  int* slev = smeta + nr + 1;
  int16_t* srow = (int16_t*)(slev + nlev + 1);
  int16_t* scol = srow + nr;
  int16_t* sT = scol + ne;
  const int t = threadIdx.x, nt = blockDim.x;
  const int ntile = nr * TW;
  // metadata.  Per level position: the row, and its first entry | length <<
  // 20 (entries of a pack below 2^20, row lengths below 2^11: checked on the
  // host), so that both come from one LDS round trip.  The first pass of
  // every array (column indices and values eight per thread, tail rows,
  // program rows, level bounds) is loaded at once, then the row bounds that
  // depend on the program rows, then everything is stored: two memory round
  // trips; items past one pass (packs larger than the workgroup) follow.
  {
    int16_t cv[8];
    double pv[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = min(t + m * nt, ne - 1);
      cv[m] = ne > 0 ? ecol[e0 + e] : (int16_t)0;
      if (SV) pv[m] = ne > 0 ? pval[e0 + e] : 0.0;
    }
    const int16_t tv = nT > 0 ? trows[tq + min(t, nT - 1)] : (int16_t)0;
    const int lr = nprog > 0 ? lrows[base_row + min(t, nprog - 1)] : r0;
    const int lvv = lev[l0 + min(t, nlev)];
    const int row = lr - r0;
    const int es = rp[r0 + row], ee = rp[r0 + row + 1];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = t + m * nt;
      if (e < ne) {
        scol[e] = cv[m];
        if (SV) sval[e] = pv[m];
      }
    }
    if (t < nT) sT[t] = tv;
    if (t < nprog) {
      srow[t] = (int16_t)row;
      smeta[t] = (es - e0) | ((ee - es) << 20);
    }
    if (t <= nlev) slev[t] = lvv - base_row;
  }
  for (int eb = t + 8 * nt; eb < ne; eb += 8 * nt) {
    int16_t cv[8];
    double pv[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = min(eb + m * nt, ne - 1);
      cv[m] = ecol[e0 + e];
      if (SV) pv[m] = pval[e0 + e];
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = eb + m * nt;
      if (e < ne) {
        scol[e] = cv[m];
        if (SV) sval[e] = pv[m];
      }
    }
  }
  for (int k = t + nt; k < nT; k += nt) sT[k] = trows[tq + k];
  for (int p = t + nt; p < nprog; p += nt) {
    const int row = lrows[base_row + p] - r0;
    const int es = rp[r0 + row], ee = rp[r0 + row + 1];
    srow[p] = (int16_t)row;
    smeta[p] = (es - e0) | ((ee - es) << 20);
  }
  for (int k = t + nt; k <= nlev; k += nt) slev[k] = lev[l0 + k] - base_row;
  if (FWD && fz.jp) {
    // right-hand side R = -J_u V formed here from the directions V (rows of
    // J_u over the pack's rows, a few entries each): eight elements per
    // thread at a time, each round of loads (row bounds, entries, V) issued
    // for all eight before any is used
    for (int eb = t; eb < ntile; eb += 8 * nt) {
      int pa[8], pb[8], cc[8];
      int kmax = 0;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int e = min(eb + m * nt, ntile - 1);
        const int r = e / TW;
        cc[m] = min(c0 + (e - r * TW), ncols - 1);
        pa[m] = fz.jp[r0 + r];
        pb[m] = fz.jp[r0 + r + 1];
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) kmax = max(kmax, pb[m] - pa[m]);
      double acc[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) acc[m] = 0.0;
      for (int k = 0; k < kmax; ++k) {
        double jv[8];
        int jc[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int pp = min(pa[m] + k, max(pb[m] - 1, pa[m]));
          jv[m] = pa[m] + k < pb[m] ? fz.jv[pp] : 0.0;
          jc[m] = pa[m] + k < pb[m] ? fz.jc[pp] : 0;
        }
        double vv[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) vv[m] = fz.V[(size_t)jc[m] * fz.ldv + cc[m]];
#pragma unroll
        for (int m = 0; m < 8; ++m) acc[m] += jv[m] * vv[m];
      }
#pragma unroll
      for (int m = 0; m < 8; ++m)
        if (eb + m * nt < ntile) xs[eb + m * nt] = -scale * acc[m];
    }
  } else {
    // right-hand-side tile, eight loads in flight per thread
    for (int eb = t; eb < ntile; eb += 8 * nt) {
      double v[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int e = min(eb + m * nt, ntile - 1);
        const int r = e / TW, c = e - r * TW;
        v[m] = X[(size_t)(r0 + r) * ld + min(c0 + c, ncols - 1)];
      }
#pragma unroll
      for (int m = 0; m < 8; ++m)
        if (eb + m * nt < ntile) xs[eb + m * nt] = FWD ? scale * v[m] : v[m];
    }
  }
  __syncthreads();
  if (!FWD && fz.tmoff) {
    // backward: the products of the pack rows that have entries in top
    // columns with the solved top part, subtracted here (one thread per row
    // and column; a row's entries eight at a time, all their loads issued
    // before the first is used, summed in entry order)
    const int a0 = fz.tmoff[q], na = fz.tmoff[q + 1] - a0;
    for (int e = t; e < na * TW; e += nt) {
      const int rr = e / TW, c = e - rr * TW;
      const int i = fz.tmrows[a0 + rr];
      const int cc = min(c0 + c, ncols - 1);
      const int pa = up_split[i], pb = ptr[i + 1];
      double acc = 0.0;
      for (int pp = pa; pp < pb; pp += 8) {
        double vv[8], xv[8];
        int cl[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int pm = min(pp + m, pb - 1);
          vv[m] = pp + m < pb ? val[pm] : 0.0;
          cl[m] = col[pm];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) xv[m] = X[(size_t)cl[m] * ld + cc];
#pragma unroll
        for (int m = 0; m < 8; ++m) acc += vv[m] * xv[m];
      }
      xs[(i - r0) * TW + c] -= acc;
    }
    __syncthreads();
  }
  const double* Mq = tinv + (size_t)q * TAIL_MAX * TAIL_MAX;
  // backward: the tail rows first, by the dense inverse of U_TT (or L_TT^T)
  if (!FWD && nT > 0) tail_apply_any<TW>(xs, sT, nT, Mq, false);
  const int wave = t >> 6, lane = t & 63, nwave = nt >> 6;
  const int cI = lane & (TW - 1);
  const int sub = lane / TW;   // 0 .. S - 1
  for (int lv = 0; lv < nlev; ++lv) {
    const int a = slev[lv], nrow = slev[lv + 1] - a;
    // forward: the last level holds the tail rows, gathering only their
    // entries outside the tail (no pivot: the dense inverse has it)
    const bool gather = FWD && nT > 0 && lv == nlev - 1;
    // R = 2^lgR rows per wavefront, G = S / R lanes per (row, column)
    int lgR = LGS;
    while (lgR > 0 && nrow <= (nwave << (lgR - 1))) --lgR;
    const int lgG = LGS - lgR;
    const int G = 1 << lgG;
    const int rowslot = sub >> lgG, seg = sub & (G - 1);
    for (int base = 0; base < nrow; base += nwave << lgR) {
      const int k = base + (wave << lgR) + rowslot;
      const bool act = k < nrow;
      const int kk = a + min(k, nrow - 1);
      const int rl = srow[kk];
      const int meta = smeta[kk];
      // the row's own right-hand side (no other row writes it) and pivot
      // reciprocal, loaded before the entry loop, off the chain that ends
      // in the row's store
      const double xo = xs[rl * TW + cI];
      const double rdv = UNIT ? 1.0 : rdg[r0 + rl];
      double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
      if (act) {
        const int es = meta & 0xFFFFF, ee = es + (meta >> 20);
        for (int eb = es + seg; eb < ee; eb += 8 * G) {
          double vv[8], xv[8];
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            const int e = eb + m * G;
            const bool in = e < ee;
            const int ec = in ? e : es;
            const double raw = SV ? sval[ec] : pval[e0 + ec];
            vv[m] = in ? raw : 0.0;
            xv[m] = xs[scol[ec] * TW + cI];
          }
          q0 += vv[0] * xv[0] + vv[4] * xv[4];
          q1 += vv[1] * xv[1] + vv[5] * xv[5];
          q2 += vv[2] * xv[2] + vv[6] * xv[6];
          q3 += vv[3] * xv[3] + vv[7] * xv[7];
        }
      }
      double part = (q0 + q1) + (q2 + q3);
      if (TW == 16) {   // lanes c, c + 16, c + 32, c + 48 share column c
        if (G >= 4) part = sum_xor32(part);
        if (G >= 2) part = sum_xor16(part);
      } else {
        for (int o = G >> 1; o > 0; o >>= 1) part += __shfl_xor(part, o * TW, 64);
      }
      if (act && seg == 0) {
        double v = xo - part;
        if (!UNIT && !gather) v *= rdv;
        xs[rl * TW + cI] = v;
      }
    }
    lds_barrier();
  }
  // forward: the tail rows by the dense inverse of L_TT (or U_TT^T)
  if (FWD && nT > 0) tail_apply_any<TW>(xs, sT, nT, Mq, true);
  for (int e = t; e < ntile; e += nt) {
    const int r = e / TW, c = e - r * TW;
    if (c0 + c < ncols) X[(size_t)(r0 + r) * ld + c0 + c] = xs[e];
  }
}

// Dense T x T blocks of the pack tails from the LU values: A[q][0] = L_TT
// (unit diagonal), A[q][1] = U_TT, row-major with leading dimension
// TAIL_MAX, zero elsewhere (k_fill_dbl first).  One thread per entry.
__global__ void k_tail_gather(int ne, const int32_t* __restrict__ eoff, int npacks, const int32_t* __restrict__ pos,
                              const int32_t* __restrict__ dense, const int32_t* __restrict__ toff,
                              const double* __restrict__ luv, double* __restrict__ A,
                              const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) {
    int lo = 0, hi = npacks;   // pack of entry e: eoff[q] <= e < eoff[q + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (eoff[mid] <= e) lo = mid;
      else hi = mid;
    }
    const int q = lo;
    const int d = dense[e];
    const int a = d / TAIL_MAX, b = d - a * TAIL_MAX;
    double* Aq = A + (size_t)q * 2 * TAIL_MAX * TAIL_MAX;
    if (b < a) Aq[d] = luv[pos[e]];
    else Aq[TAIL_MAX * TAIL_MAX + d] = luv[pos[e]];
    if (a == b) Aq[d] = 1.0;
  }
}

// Inverses of the tail blocks in 64 x 64 blocks (a tail has at most two):
// k_tail_diag_inv inverts the diagonal blocks of L_TT (unit) and U_TT, one
// workgroup per (pack, part, block), as k_top_diag_inv does for the top;
// k_tail_offdiag then forms the off-diagonal block of each inverse,
//   (L^-1)_21 = -L22^-1 (L21 L11^-1),  (U^-1)_12 = -U11^-1 (U12 U22^-1).
// Out: Minv[0] = L_TT^-1, [1] = U_TT^-1, [2] = (L_TT^-1)^T, [3] =
// (U_TT^-1)^T, each [npacks][TAIL_MAX x TAIL_MAX] (entries past nT are
// never read).
__global__ void __launch_bounds__(256) k_tail_diag_inv(const int32_t* __restrict__ toff, const double* __restrict__ A,
                                                       double* __restrict__ Minv, int npacks,
                                                       const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double T[CB][CB + 1];
  __shared__ double rd[CB];
  const int q = blockIdx.x, part = blockIdx.y, kb = blockIdx.z;
  const int nT = toff[q + 1] - toff[q];
  const int b0 = kb * CB;
  if (b0 >= nT) return;
  const int nb = min(CB, nT - b0);
  const double* Aq = A + ((size_t)q * 2 + part) * TAIL_MAX * TAIL_MAX;
  const int t = threadIdx.x;
  {
    double v[CB * CB / 256];
#pragma unroll
    for (int m = 0; m < CB * CB / 256; ++m) {
      const int e = t + 256 * m, r = e >> 6, cc = e & 63;
      v[m] = Aq[(size_t)(b0 + min(r, nb - 1)) * TAIL_MAX + b0 + min(cc, nb - 1)];
    }
#pragma unroll
    for (int m = 0; m < CB * CB / 256; ++m) {
      const int e = t + 256 * m, r = e >> 6, cc = e & 63;
      const bool in = r < nb && cc < nb && (part == 0 ? cc < r : cc > r);
      T[r][cc] = in ? v[m] : 0.0;
    }
  }
  if (t < CB) rd[t] = (part == 0 || t >= nb) ? 1.0 : 1.0 / Aq[(size_t)(b0 + t) * TAIL_MAX + b0 + t];
  __syncthreads();
  const int c = t >> 2, seg = t & 3;
  double zr[CB / 4];
#pragma unroll
  for (int m = 0; m < CB / 4; ++m) zr[m] = 0.0;
  if (part == 0) tri_inv_rows<true>(T, rd, c, seg, nb, zr);
  else tri_inv_rows<false>(T, rd, c, seg, nb, zr);
  const size_t blk = (size_t)TAIL_MAX * TAIL_MAX, n4 = (size_t)npacks * blk;
  double* Mo = Minv + (size_t)part * n4 + (size_t)q * blk;
  double* Mt = Minv + (size_t)(2 + part) * n4 + (size_t)q * blk;
#pragma unroll
  for (int m = 0; m < CB / 4; ++m) {
    const int r = b0 + 4 * m + seg, cc = b0 + c;
    Mo[(size_t)r * TAIL_MAX + cc] = zr[m];
    Mt[(size_t)cc * TAIL_MAX + r] = zr[m];
  }
}

// Off-diagonal blocks of the tail inverses (tails longer than CB rows):
// part 0, rows CB .. nT of L^-1: X21 = -D2 (L21 D1); part 1, columns CB ..
// nT of U^-1: Y12 = -E1 (U12 E2), with D1, D2, E1, E2 the diagonal-block
// inverses from k_tail_diag_inv.  One workgroup (256 threads) per (pack,
// part): the operands pass through two 64 x 64 LDS blocks; thread (tr, tc)
// forms the 4 x 4 register tile of rows 4 tr.., columns 4 tc.., reading
// four entries of each operand per step k.
__device__ __forceinline__ void tile_mm4(const double (*X)[CB + 1], const double (*Y)[CB + 1], int tr, int tc,
                                         double (&acc)[4][4]) {
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
#pragma unroll 4
  for (int k = 0; k < CB; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) a[p] = X[4 * tr + p][k];
#pragma unroll
    for (int q = 0; q < 4; ++q) b[q] = Y[k][4 * tc + q];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
  }
}

__global__ void __launch_bounds__(256) k_tail_offdiag(const int32_t* __restrict__ toff, const double* __restrict__ A,
                                                      double* __restrict__ Minv, int npacks,
                                                      const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double S1[CB][CB + 1], S2[CB][CB + 1];
  const int q = blockIdx.x, part = blockIdx.y;
  const int nT = toff[q + 1] - toff[q];
  if (nT <= CB) return;
  const int n2 = nT - CB;
  const size_t blk = (size_t)TAIL_MAX * TAIL_MAX, n4 = (size_t)npacks * blk;
  const double* Aq = A + ((size_t)q * 2 + part) * blk;
  double* Mo = Minv + (size_t)part * n4 + (size_t)q * blk;
  double* Mt = Minv + (size_t)(2 + part) * n4 + (size_t)q * blk;
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  // part 0: S1 = L21 (n2 x CB), S2 = D1 (CB x CB); part 1: S1 = U12
  // (CB x n2), S2 = E2 (n2 x n2)
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, cc = e & 63;
    if (part == 0) {
      S1[r][cc] = r < n2 ? Aq[(size_t)(CB + r) * TAIL_MAX + cc] : 0.0;
      S2[r][cc] = Mo[(size_t)r * TAIL_MAX + cc];
    } else {
      S1[r][cc] = cc < n2 ? Aq[(size_t)r * TAIL_MAX + CB + cc] : 0.0;
      S2[r][cc] = (r < n2 && cc < n2) ? Mo[(size_t)(CB + r) * TAIL_MAX + CB + cc] : 0.0;
    }
  }
  __syncthreads();
  double acc[4][4];
  tile_mm4(S1, S2, tr, tc, acc);
  __syncthreads();
  // S1 = the product, S2 = D2 (part 0) or E1 (part 1)
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) S1[4 * tr + p][4 * tc + qq] = acc[p][qq];
  for (int e = t; e < CB * CB; e += 256) {
    const int r = e >> 6, cc = e & 63;
    if (part == 0) S2[r][cc] = (r < n2 && cc < n2) ? Mo[(size_t)(CB + r) * TAIL_MAX + CB + cc] : 0.0;
    else S2[r][cc] = Mo[(size_t)r * TAIL_MAX + cc];
  }
  __syncthreads();
  // part 0: X21 = -D2 S1 (n2 x CB); part 1: Y12 = -E1 S1 (CB x n2)
  tile_mm4(S2, S1, tr, tc, acc);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int r = 4 * tr + p, cc = 4 * tc + qq;
      const double v = -acc[p][qq];
      if (part == 0) {
        if (r < n2) {
          Mo[(size_t)(CB + r) * TAIL_MAX + cc] = v;
          Mt[(size_t)cc * TAIL_MAX + CB + r] = v;
        }
      } else if (cc < n2) {
        Mo[(size_t)r * TAIL_MAX + CB + cc] = v;
        Mt[(size_t)(CB + cc) * TAIL_MAX + r] = v;
      }
    }
}

// ------------------------------------------------------------------ SpMM
// One CSR term sum_p v(p) * s(col) * X[col, c] of a sparse-dense product,
// with v(p) = val[valpos ? valpos[p] : p], s = xscale ? xscale[col] : 1.
struct SpTerm {
  const int32_t* ptr;
  const int32_t* col;
  const double* val;
  const int32_t* valpos;
  const double* xscale;
  const double* X;
  int ldx;
};

// Row i of a term for columns c0 + 64 m (m < CPT) of one lane: the row's
// entries are the same in every lane of the wavefront (i uniform), so they
// are read as scalars.  Eight entries per pass with all their X loads in
// flight (addresses clamped, padding entries weighted 0); entry p adds into
// partial sum (p - p0) mod 4, combined as (s0 + s1) + (s2 + s3).
template <int CPT>
__device__ __forceinline__ void spmm_row(const SpTerm& A, int i, int c0, int ncols, double (&r)[CPT]) {
  const int p0 = A.ptr[i], p1 = A.ptr[i + 1];
  double a[CPT][4];
#pragma unroll
  for (int k = 0; k < CPT; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) a[k][m] = 0.0;
  for (int pb = p0; pb < p1; pb += 8) {
    int jj[8];
    double vv[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int pc = min(pb + m, p1 - 1);
      jj[m] = A.col[pc];
      const double raw = A.val[A.valpos ? A.valpos[pc] : pc];
      vv[m] = pb + m < p1 ? raw : 0.0;
    }
    if (A.xscale) {
#pragma unroll
      for (int m = 0; m < 8; ++m) vv[m] *= A.xscale[jj[m]];
    }
    double xv[8][CPT];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
      for (int k = 0; k < CPT; ++k) xv[m][k] = A.X[(size_t)jj[m] * A.ldx + min(c0 + 64 * k, ncols - 1)];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
      for (int k = 0; k < CPT; ++k) a[k][m & 3] += vv[m] * xv[m][k];
  }
#pragma unroll
  for (int k = 0; k < CPT; ++k) r[k] = (a[k][0] + a[k][1]) + (a[k][2] + a[k][3]);
}

// Y[i, c] = alpha * (A1 row i)(c) (+ Yadd[i, c]); with TWO, then
// Y[i, c] = alpha2 * (A2 row i)(c) + that.  One wavefront per row, lane l
// taking columns c0 + l + 64 m (m < CPT); 256 threads, four rows per
// workgroup.
template <int CPT, bool TWO>
__global__ void __launch_bounds__(256) k_spmm(int nrows, SpTerm A1, SpTerm A2, int ncols, double alpha, double alpha2,
                                              const double* __restrict__ Yadd, int ldya, double* __restrict__ Y,
                                              int ldy, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (int)(threadIdx.x >> 6));
  if (i >= nrows) return;
  const int lane = threadIdx.x & 63;
  const int c0 = blockIdx.x * 64 * CPT + lane;
  double r[CPT], r2[CPT];
  spmm_row<CPT>(A1, i, c0, ncols, r);
  if (TWO) spmm_row<CPT>(A2, i, c0, ncols, r2);
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = c0 + 64 * k;
    if (c < ncols) {
      double acc = r[k] * alpha;
      if (Yadd) acc += Yadd[(size_t)i * ldya + c];
      if (TWO) acc = r2[k] * alpha2 + acc;
      Y[(size_t)i * ldy + c] = acc;
    }
  }
}

__global__ void k_copy_block(int n, int ncols, const double* __restrict__ src, int lds_,
                             double* __restrict__ dst, int ldd, const int32_t* __restrict__ skip = nullptr) {
  if (skip && *skip) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i < n && c < ncols) dst[(size_t)i * ldd + c] = src[(size_t)i * lds_ + c];
}

// identity columns j0 .. j0 + ncols - 1 of an n x n identity, as [n x ncols]
__global__ void k_identity_block(int n, int ncols, int j0, double* __restrict__ dst, int ldd,
                                 const int32_t* __restrict__ skip = nullptr) {
  if (skip && *skip) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i < n && c < ncols) dst[(size_t)i * ldd + c] = (i == j0 + c) ? 1.0 : 0.0;
}

// ----------------------------------------------- AL constraints, weights
struct ALArgs {
  int nb, nl, npq, npv, ng, m, nx, nu;
  int ref, gen_ref;
  double base, rho;
  const double* sigf;       // [1] sigma_f (device)
  const int32_t* pq;        // [npq]
  const int32_t* pv;        // [npv]
  const int32_t* gen_pidx;  // [ng] control index of p_g (PV), -1 for the slack
  const int32_t* pv_gen;    // [npv] generator at each PV bus
  const double* c2;
  const double* c1;
  const double* c0;
  const double* rec;        // branch records
  const double* Pbus;       // [nb] bus injections P_i
  const double* Qbus;       // [nb]
  const double* vm;         // [nb]
  const double* pd;
  const double* qd;
  const double* u;
  const double* s;          // [m]
  const double* y;          // [m]
  const double* sigma_c;    // [m]
};

// c_k, the AL weight w_k = d phi / d c_k and the phi term of constraint k
// (terms[k]); generator cost terms sigma_f f_g in terms[m + g].
__global__ void k_constraints(ALArgs A, double* __restrict__ c, double* __restrict__ w,
                              double* __restrict__ terms) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < A.m) {
    double ck;
    if (k < A.nl) {
      const double* o = A.rec + (size_t)k * RECW;
      ck = o[0] * o[0] + o[1] * o[1];
    } else if (k < 2 * A.nl) {
      const double* o = A.rec + (size_t)(k - A.nl) * RECW;
      ck = o[2] * o[2] + o[3] * o[3];
    } else if (k < 2 * A.nl + A.npq) {
      ck = A.vm[A.pq[k - 2 * A.nl]];
    } else if (k == 2 * A.nl + A.npq) {
      ck = A.Pbus[A.ref] + A.pd[A.ref];
    } else if (k == 2 * A.nl + A.npq + 1) {
      ck = A.Qbus[A.ref] + A.qd[A.ref];
    } else {
      const int b = A.pv[k - 2 * A.nl - A.npq - 2];
      ck = A.Qbus[b] + A.qd[b];
    }
    const double sc = A.sigma_c[k];
    const double r = sc * (ck - A.s[k]);
    if (c) c[k] = ck;
    if (w) w[k] = sc * (A.y[k] + A.rho * r);
    if (terms) terms[k] = A.y[k] * r + 0.5 * A.rho * r * r;
  } else if (k < A.m + A.ng) {
    const int gi = k - A.m;
    const double p = gi == A.gen_ref ? A.Pbus[A.ref] + A.pd[A.ref] : A.u[A.gen_pidx[gi]];
    const double pm = A.base * p;
    if (terms) terms[k] = A.sigf[0] * (A.c2[gi] * pm * pm + A.c1[gi] * pm + A.c0[gi]);
  }
}

// Weights of the bus injections in l = phi + lambda^T g: a_i on P_i and
// b_i on Q_i (lambda may be null); threads past nb fill the rank-one
// coefficients kappa of (p_ref, q_ref, q_pv): the constraint's curvature
// weight rho sigma_k^2, or gn[k] when gn is given (the Schur-complement
// weights of the bounded QP), plus the slack's cost curvature for p_ref.
__global__ void k_bus_weights(ALArgs A, const double* __restrict__ w, const double* __restrict__ lam,
                              const int32_t* __restrict__ rowP, const int32_t* __restrict__ rowQ,
                              const int32_t* __restrict__ bus_pvpos, double* __restrict__ a,
                              double* __restrict__ b, double* __restrict__ kappa,
                              const double* __restrict__ gn = nullptr,
                              const int32_t* __restrict__ skip = nullptr) {
  if (skip && *skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int kp = 2 * A.nl + A.npq;
  const double sigma_f = A.sigf[0];
  if (i < A.nb) {
    double ai = 0.0, bi = 0.0;
    if (lam) {
      if (rowP[i] >= 0) ai += lam[rowP[i]];
      if (rowQ[i] >= 0) bi += lam[rowQ[i]];
    }
    if (i == A.ref) {
      const double pref = A.Pbus[A.ref] + A.pd[A.ref];
      const int gr = A.gen_ref;
      ai += sigma_f * A.base * (2.0 * A.c2[gr] * A.base * pref + A.c1[gr]) + w[kp];
      bi += w[kp + 1];
    }
    const int pp = bus_pvpos[i];
    if (pp >= 0) bi += w[kp + 2 + pp];
    a[i] = ai;
    b[i] = bi;
  } else if (i < A.nb + 2 + A.npv) {
    const int r = i - A.nb;
    const double sc = A.sigma_c[kp + r];
    double kap = gn ? gn[kp + r] : A.rho * sc * sc;
    if (r == 0) kap += sigma_f * 2.0 * A.c2[A.gen_ref] * A.base * A.base;
    kappa[r] = kap;
  }
}

// Second-order branch records: for l = sum_e (a P_e + b Q_e + w_h h_e) +
// rho/2 (sigma_h h_e)^2-type curvature, the local gradient (4) and the
// local 4x4 Hessian W in (theta_f, theta_t, v_f, v_t):
//   alpha_e = a + 2 w_h P_e, beta_e = b + 2 w_h Q_e,
//   W = sum_e d2(alpha_e P_e + beta_e Q_e) + 2 w_h (dP dP^T + dQ dQ^T)
//       + kappa_h dh dh^T,  dh = 2 P dP + 2 Q dQ,  kappa_h = rho sigma_h^2
// (gn[k] instead when gn is given).
__global__ void k_branch_second(int nl, const int32_t* __restrict__ bf, const int32_t* __restrict__ bt,
                                const double* __restrict__ br, const double* __restrict__ bx,
                                const double* __restrict__ bb, const double* __restrict__ th,
                                const double* __restrict__ vm, const double* __restrict__ rec,
                                const double* __restrict__ a, const double* __restrict__ b,
                                const double* __restrict__ w, const double* __restrict__ sigma_c,
                                double rho, double* __restrict__ wrec, const double* __restrict__ gn = nullptr,
                                const int32_t* __restrict__ skip = nullptr) {
  if (skip && *skip) return;
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  const int f = bf[l], t = bt[l];
  const double r = br[l], x = bx[l], bsh = 0.5 * bb[l];
  const double z2 = r * r + x * x;
  const double gs = r / z2, bs = -x / z2;
  const double Goo = gs, Boo = bs + bsh, Gm = -gs, Bm = -bs;
  const double vf = vm[f], vt = vm[t];
  double sn, cs;
  sincos(th[f] - th[t], &sn, &cs);
  const double vv = vf * vt;
  const double Af = Gm * cs + Bm * sn, Cf = Gm * sn - Bm * cs;
  const double At = Gm * cs - Bm * sn, Ct = -Gm * sn - Bm * cs;
  const double* o = rec + (size_t)l * RECW;
  double W[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) W[i][j] = 0.0;
  double gl[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int bus = e == 0 ? f : t;
    const int kc = e == 0 ? l : nl + l;
    const double wh = w[kc];
    const double sh = sigma_c[kc];
    const double P = o[2 * e], Q = o[2 * e + 1];
    const double* dP = o + 4 + 8 * e;
    const double* dQ = o + 8 + 8 * e;
    const double al = a[bus] + 2.0 * wh * P;
    const double be = b[bus] + 2.0 * wh * Q;
    // second derivatives of al * P_e + be * Q_e
    double T, Tp, K;
    if (e == 0) {
      T = al * Af + be * Cf;
      Tp = -al * Cf + be * Af;
      K = al * Goo - be * Boo;
    } else {
      T = al * At + be * Ct;
      Tp = al * Ct - be * At;
      K = al * Goo - be * Boo;
    }
    W[0][0] += -vv * T;
    W[1][1] += -vv * T;
    W[0][1] += vv * T;
    W[0][2] += vt * Tp;
    W[0][3] += vf * Tp;
    W[1][2] += -vt * Tp;
    W[1][3] += -vf * Tp;
    W[2][3] += T;
    W[2 + e][2 + e] += 2.0 * K;
    const double kap = gn ? gn[kc] : rho * sh * sh;
    double dh[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dh[i] = 2.0 * (P * dP[i] + Q * dQ[i]);
      gl[i] += al * dP[i] + be * dQ[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i; j < 4; ++j)
        W[i][j] += 2.0 * wh * (dP[i] * dP[j] + dQ[i] * dQ[j]) + kap * dh[i] * dh[j];
  }
  double* q = wrec + (size_t)l * WREC;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) q[4 * i + j] = i <= j ? W[i][j] : W[j][i];
#pragma unroll
  for (int i = 0; i < 4; ++i) q[16 + i] = gl[i];
}

// Gradient of the (Lagrangian) function over all variables: gathered
// branch-local gradients plus the terms not carried by branches:
// v_pq: w of the voltage constraint; p_pv: sigma_f f'(p) - lambda_P.
struct VarArgs {
  int nvar, nx, npq, npv, nl;
  double base;
  const double* sigf;    // [1] sigma_f (device)
  const int32_t* kind;   // 0 theta, 1 v_pq, 2 v control, 3 p_pv
  const int32_t* aux;    // v_pq: pq position; p_pv: pv position
  const int32_t* pv_gen;
  const int32_t* pv;
  const int32_t* rowP;
  const double* c2;
  const double* c1;
  const double* u;
};

__global__ void k_var_grad(VarArgs V, const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
                           const double* __restrict__ wrec, const double* __restrict__ w,
                           const double* __restrict__ lam, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= V.nvar) return;
  double acc = 0.0;
  for (int j = ptr[c]; j < ptr[c + 1]; ++j) acc += wrec[src[j]];
  const int kd = V.kind[c];
  if (kd == 1) {
    acc += w[2 * V.nl + V.aux[c]];
  } else if (kd == 3) {
    const int k = V.aux[c];
    const int gi = V.pv_gen[k];
    const double p = V.u[1 + V.npv + k];
    acc += V.sigf[0] * V.base * (2.0 * V.c2[gi] * V.base * p + V.c1[gi]);
    if (lam) acc -= lam[V.rowP[V.pv[k]]];
  }
  out[c] = acc;
}

// Diagonal terms of K not carried by branches: rho sigma_v^2 (gn[k] when
// gn is given) on v_pq and the PV cost curvature sigma_f 2 c2 B^2 on p_pv.
__global__ void k_k_diag(VarArgs V, const int32_t* __restrict__ kdiag, const double* __restrict__ sigma_c,
                         double rho, double* __restrict__ kval, const double* __restrict__ gn = nullptr,
                         const int32_t* __restrict__ skip = nullptr) {
  if (skip && *skip) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= V.nvar) return;
  const int kd = V.kind[c];
  if (kd == 1) {
    const int k = 2 * V.nl + V.aux[c];
    const double sv = sigma_c[k];
    kval[kdiag[c]] += gn ? gn[k] : rho * sv * sv;
  } else if (kd == 3) {
    const int gi = V.pv_gen[V.aux[c]];
    kval[kdiag[c]] += V.sigf[0] * 2.0 * V.c2[gi] * V.base * V.base;
  }
}

__global__ void k_axpy(int n, double a, const double* __restrict__ x, double* __restrict__ y,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// Reduced Jacobian of the constraints for a batch of directions (Section
// III-C): J[k][j0 + col] = grad c_k . D[:, col], with D = [Z; V] over all
// variables (internal order), i.e. (d_x c) Z + d_u c.  Rows: h at the from
// and to ends through the branch records (d|S|^2 = 2 (P dP + Q dQ) over
// theta_f, theta_t, v_f, v_t), v at the PQ buses (a state row of D), and
// p_ref, q_ref, q_pv from T = G D (the rank-one rows, rows of T in that
// order).  Threads (64, 4): the batch's columns along the lanes.
__global__ void k_cjac_batch(int nl, int npq, int m, int B, const int32_t* __restrict__ br_f,
                             const int32_t* __restrict__ br_t, const int32_t* __restrict__ th_var,
                             const int32_t* __restrict__ v_var, const int32_t* __restrict__ pq,
                             const double* __restrict__ rec, const double* __restrict__ D, int ldd,
                             const double* __restrict__ T, int ldt, double* __restrict__ J, int ldj, int j0) {
  const int col = blockIdx.x * 64 + threadIdx.x;
  const int k = blockIdx.y * 4 + threadIdx.y;
  if (k >= m || col >= B) return;
  double v;
  if (k < 2 * nl) {
    const int e = k >= nl ? 1 : 0;
    const int l = k - e * nl;
    const double* o = rec + (size_t)l * RECW;
    const double P = o[2 * e], Q = o[2 * e + 1];
    const double* dP = o + 4 + 8 * e;
    const double* dQ = dP + 4;
    const int f = br_f[l], t = br_t[l];
    const int var[4] = {th_var[f], th_var[t], v_var[f], v_var[t]};
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (var[q] >= 0) acc += (P * dP[q] + Q * dQ[q]) * D[(size_t)var[q] * ldd + col];
    v = 2.0 * acc;
  } else if (k < 2 * nl + npq) {
    v = D[(size_t)v_var[pq[k - 2 * nl]] * ldd + col];
  } else {
    v = T[(size_t)(k - 2 * nl - npq) * ldt + col];
  }
  J[(size_t)k * ldj + j0 + col] = v;
}

// pivot words of the refactorizations (piv[0]: sparse rows, piv[1]: dense
// top block; internal row + 1) as a 1-based index in the paper's x order,
// 0 when every pivot passed
__device__ __forceinline__ int32_t pivot_report(const int32_t* __restrict__ piv, const int32_t* __restrict__ x_i2p) {
  const int32_t r = piv[0] != 0 ? piv[0] : piv[1];
  return r > 0 ? x_i2p[r - 1] + 1 : 0;
}

// power-flow status {Newton steps, converged, tiny pivot} and residual
__global__ void k_pf_status(int32_t* __restrict__ st, const int32_t* __restrict__ count,
                            const int32_t* __restrict__ done, const int32_t* __restrict__ piv,
                            const int32_t* __restrict__ x_i2p, const double* __restrict__ rsrc,
                            double* __restrict__ rdst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st[0] = count[0];
    st[1] = done[0] == 1 ? 1 : 0;
    st[2] = pivot_report(piv, x_i2p);
    rdst[0] = rsrc[0];
  }
}

__global__ void k_piv_report(const int32_t* __restrict__ piv, const int32_t* __restrict__ x_i2p,
                             int32_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = pivot_report(piv, x_i2p);
}

__global__ void k_fill_int(int n, int32_t* __restrict__ p, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// --------------------------------------------------------- tracking step
__global__ void k_copy_vec(int n, const double* __restrict__ src, double* __restrict__ dst,
                           const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_neg_copy(int n, const double* __restrict__ src, double* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = -src[i];
}

__global__ void k_count(const int32_t* __restrict__ skip, int32_t* __restrict__ count) {
  if (skip && *skip) return;
  if (threadIdx.x == 0 && blockIdx.x == 0) count[0] += 1;
}

__global__ void k_copy_int(const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

// loads of one tracking step: base loads times per-bus factors
__global__ void k_track_loads(int nb, const double* __restrict__ pd0, const double* __restrict__ qd0,
                              const double* __restrict__ fac, double* __restrict__ pd, double* __restrict__ qd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) {
    pd[i] = pd0[i] * fac[i];
    qd[i] = qd0[i] * fac[i];
  }
}

// closed-form minimiser of the scaled AL in s: clip(c + y / (rho sigma_c))
__global__ void k_slack(int m, const double* __restrict__ c, const double* __restrict__ y,
                        const double* __restrict__ sigma_c, double rho, const double* __restrict__ lo,
                        const double* __restrict__ hi, double* __restrict__ s) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) s[k] = fmin(fmax(c[k] + y[k] / (rho * sigma_c[k]), lo[k]), hi[k]);
}

// multiplier update with the slack minimiser at the new point:
// s = clip(c + y / (rho sigma)), y += rho sigma (c - s)
__global__ void k_y_update(int m, const double* __restrict__ c, const double* __restrict__ sigma_c, double rho,
                           const double* __restrict__ lo, const double* __restrict__ hi, double* __restrict__ y,
                           double* __restrict__ s) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) {
    const double sk = fmin(fmax(c[k] + y[k] / (rho * sigma_c[k]), lo[k]), hi[k]);
    s[k] = sk;
    y[k] = y[k] + rho * sigma_c[k] * (c[k] - sk);
  }
}

// trial control u + f d clipped to the control bounds
__global__ void k_try_u(int n, const double* __restrict__ u, const double* __restrict__ d, double f,
                        const double* __restrict__ lo, const double* __restrict__ hi, double* __restrict__ ut,
                        const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ut[i] = fmin(fmax(u[i] + f * d[i], lo[i]), hi[i]);
}

// v *= a
__global__ void k_scale_vec(int n, double a, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] *= a;
}

// trial point of the exact step: ut = u + f du, st = s + f ds (the QP's box
// keeps both inside their bounds; no clipping)
__global__ void k_try_w(int nu, int m, const double* __restrict__ u, const double* __restrict__ sv,
                        const double* __restrict__ dw, double f, double* __restrict__ ut, double* __restrict__ st,
                        const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nu) ut[i] = u[i] + f * dw[i];
  else if (i < nu + m) st[i - nu] = sv[i - nu] + f * dw[i];
}

// accept the trial point (u, s) when its power flow converged
__global__ void k_accept_w(int nu, int m, const double* __restrict__ resid, double tol,
                           int32_t* __restrict__ accepted, const double* __restrict__ ut,
                           const double* __restrict__ st, double* __restrict__ u, double* __restrict__ sv,
                           int32_t attempt, int32_t* __restrict__ which) {
  __shared__ int ok;
  if (threadIdx.x == 0) ok = (accepted[0] == 0 && resid[0] < tol) ? 1 : 0;
  __syncthreads();
  if (!ok) return;
  for (int i = threadIdx.x; i < nu + m; i += blockDim.x) {
    if (i < nu) u[i] = ut[i];
    else sv[i - nu] = st[i - nu];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    accepted[0] = 1;
    which[0] = attempt;
  }
}

// multiplier update of the exact step (Section IV-C, step 3):
// y += rho sigma_c (c - s)
__global__ void k_y_update_s(int m, const double* __restrict__ c, const double* __restrict__ sigma_c, double rho,
                             const double* __restrict__ sv, double* __restrict__ y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) y[k] = y[k] + rho * sigma_c[k] * (c[k] - sv[k]);
}

// status of the exact tracking step from the step's flags (f) and the QP's
// words (q = done, iterations): {first power flow converged, accepted
// halving (-1 none), QP iterations, QP converged, Cholesky info of the
// Schur complement, Newton steps of the first power flow, tiny pivot word
// of the factorization behind the QP data, QP stop word}
__global__ void k_track_qp_status(const int32_t* __restrict__ f, const int32_t* __restrict__ q,
                                  int32_t* __restrict__ st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int dn = q[0];
    st[0] = f[5] == 1 ? 1 : 0;
    st[1] = f[3];
    st[2] = q[1];
    st[3] = dn == 1 ? 1 : 0;
    st[4] = dn >= 16 ? dn - 16 : (dn < 0 ? -1 : 0);
    st[5] = f[6];
    st[6] = f[7];
    st[7] = dn;
  }
}

// accept the trial control when its power flow converged: accepted = 1,
// u = ut, status = attempt index
__global__ void k_accept(int n, const double* __restrict__ resid, double tol, int32_t* __restrict__ accepted,
                         const double* __restrict__ ut, double* __restrict__ u, int32_t attempt,
                         int32_t* __restrict__ which) {
  __shared__ int ok;
  if (threadIdx.x == 0) ok = (accepted[0] == 0 && resid[0] < tol) ? 1 : 0;
  __syncthreads();
  if (!ok) return;
  for (int i = threadIdx.x; i < n; i += blockDim.x) u[i] = ut[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    accepted[0] = 1;
    which[0] = attempt;
  }
}

// status of a tracking step: first power flow converged, accepted trial
// (-1: none), Cholesky info, Newton steps of the first power flow, tiny
// pivot of the factorization behind the gradient and Hessian
__global__ void k_track_status(const int32_t* __restrict__ f, int32_t* __restrict__ st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st[0] = f[5] == 1 ? 1 : 0;
    st[1] = f[3];
    st[2] = f[4];
    st[3] = f[6];
    st[4] = f[7];
  }
}

__global__ void k_zero_if(int n, const int32_t* __restrict__ info, double* __restrict__ v) {
  if (info[0] == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = 0.0;
}

// ------------------------------------------------------------ dense step
// K = (H + H^T)/2 + diag + delta I, written to both triangles.  One
// workgroup (32 x 8 threads) per pair of 32 x 32 tiles (block row bi >=
// block column bj) and its mirror: both staged through LDS, so every global
// access runs along rows.
__global__ void k_symmetrize(int n, double* __restrict__ K, const double* __restrict__ d, double delta,
                             const int32_t* __restrict__ skip = nullptr) {
  if (skip && *skip) return;
  const int bj = blockIdx.x, bi = blockIdx.y;
  if (bj > bi) return;
  __shared__ double lo[32][33], up[32][33];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i0 = bi * 32, j0 = bj * 32;
  // lo[r][c] = K[i0 + r][j0 + c], up[r][c] = K[j0 + r][i0 + c]
  double vl[4], vu[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int r = ty + 8 * m;
    vl[m] = (i0 + r < n && j0 + tx < n) ? K[(size_t)(i0 + r) * n + j0 + tx] : 0.0;
    vu[m] = (j0 + r < n && i0 + tx < n) ? K[(size_t)(j0 + r) * n + i0 + tx] : 0.0;
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    lo[ty + 8 * m][tx] = vl[m];
    up[ty + 8 * m][tx] = vu[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int r = ty + 8 * m;
    // element (i0 + r, j0 + tx) pairs with (j0 + tx, i0 + r) = up[tx][r]
    const int i = i0 + r, j = j0 + tx;
    if (i < n && j < n) K[(size_t)i * n + j] = i == j ? lo[r][tx] + ((d ? d[i] : 0.0) + delta)
                                                     : 0.5 * (lo[r][tx] + up[tx][r]);
    // mirror tile: element (j0 + r, i0 + tx) pairs with lo[tx][r]
    const int i2 = j0 + r, j2 = i0 + tx;
    if (bi != bj && i2 < n && j2 < n) K[(size_t)i2 * n + j2] = 0.5 * (up[r][tx] + lo[tx][r]);
  }
}


// ------------------------------------------- blocked dense factorizations
// Right-looking blocked LU without pivoting (CHOL = false) or Cholesky
// (CHOL = true, lower triangle) of a row-major n x n matrix, per block of
// CB columns: diagonal block by one workgroup (diag_factor for LU,
// chol_diag_rows for Cholesky), panels one wavefront per row (and per
// column for LU), trailing update in 64 x 64 tiles on the FP64 matrix
// cores.  A failing pivot records base + (column + 1) in info[0]; later
// kernels return early.

// Diagonal block factorization with the 256 threads of the calling
// workgroup; work is LDS provided by the caller (DIAG_WORK doubles).
// Returns false when a pivot fails (info set).
//
// Thread (tr, tc) holds the 4 x 4 register tile of rows 4 tr .. 4 tr + 3,
// columns 4 tc .. 4 tc + 3.  Per diagonal tile jt: its owner factorizes it
// alone (four pivots in registers) and publishes it; the tiles below it
// (and, for LU, right of it) solve against it in registers and publish the
// result; every tile of the trailing part takes the rank-4 update.  Two
// barriers per four pivots; finished factor entries stay in the registers
// that computed them and are written from there.  A failed pivot does not
// branch: the first failing index is kept (LDS minimum) and reported after
// the loop, and the factor is then not written.
constexpr int DIAG_WORK = 16 * 16 * 2 + 20 + 2;

template <bool CHOL>
__device__ __forceinline__ bool diag_factor(int n, int b0, double* __restrict__ A, int32_t* __restrict__ info, int base,
                                            double* __restrict__ work) {
  const int nb = min(CB, n - b0);
  const int t = threadIdx.x;
  double (*colp)[16] = reinterpret_cast<double (*)[16]>(work);        // panel tile below the diagonal
  double (*rowp)[16] = reinterpret_cast<double (*)[16]>(work + 256);  // LU: panel tile right of it
  double* dt = work + 512;                                             // diagonal tile, reciprocal pivots
  int* sbad = reinterpret_cast<int*>(work + 532);
  const int tr = t >> 4, tc = t & 15;
  // direct loads (clamped addresses, all issued before use); outside the
  // nb x nb corner an identity, so the padded pivots are 1 and leave the
  // corner's factor unchanged
  double a[4][4];
  {
    double g[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        g[p][q] = A[(size_t)(b0 + min(4 * tr + p, nb - 1)) * n + b0 + min(4 * tc + q, nb - 1)];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * tr + p, c = 4 * tc + q;
        a[p][q] = (r < nb && c < nb) ? g[p][q] : (r == c ? 1.0 : 0.0);
      }
  }
  if (t == 0) *sbad = CB;
  const int njt = (nb + 3) >> 2;
  for (int jt = 0; jt < njt; ++jt) {
    if (tr == jt && tc == jt) {
      int bad = CB;
      double rd[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double d = a[k][k];
        const bool ok = CHOL ? (d > 0.0 && isfinite(d)) : (fabs(d) > 0.0 && isfinite(d));
        bad = min(bad, ok ? CB : 4 * jt + k);
        // 1 / sqrt(d) (Cholesky) or 1 / d (LU): hardware estimate and one
        // Newton step (relative error ~1e-16)
        double rp;
        if (CHOL) {
          const double y0 = __builtin_amdgcn_rsq(d);
          const double h = 0.5 * y0, g = d * y0;
          rp = fma(y0, fma(-h, g, 0.5), y0);
          a[k][k] = d * rp;
        } else {
          const double y0 = __builtin_amdgcn_rcp(d);
          rp = fma(y0, fma(-d, y0, 1.0), y0);
        }
        rd[k] = rp;
#pragma unroll
        for (int p = k + 1; p < 4; ++p) a[p][k] *= rp;
#pragma unroll
        for (int p = k + 1; p < 4; ++p)
#pragma unroll
          for (int q = k + 1; q < 4; ++q)
            if (!CHOL || q <= p) a[p][q] -= a[p][k] * (CHOL ? a[q][k] : a[k][q]);
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) dt[4 * p + q] = a[p][q];
#pragma unroll
      for (int k = 0; k < 4; ++k) dt[16 + k] = rd[k];
      if (bad < CB) atomicMin(sbad, bad);
    }
    lds_barrier();
    if (tc == jt && tr > jt) {
      // X L^T = A (Cholesky: L the factored diagonal tile) or X U = A (LU)
      double D[4][4], rd[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) D[p][q] = dt[4 * p + q];
#pragma unroll
      for (int k = 0; k < 4; ++k) rd[k] = dt[16 + k];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          double x = a[p][k];
#pragma unroll
          for (int m = 0; m < k; ++m) x -= a[p][m] * (CHOL ? D[k][m] : D[m][k]);
          a[p][k] = x * rd[k];
        }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) colp[tr][4 * p + q] = a[p][q];
    }
    if (!CHOL && tr == jt && tc > jt) {
      // L Y = A, L the unit lower part of the factored diagonal tile
      double D[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) D[p][q] = dt[4 * p + q];
#pragma unroll
      for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double y = a[k][q];
#pragma unroll
          for (int m = 0; m < k; ++m) y -= D[k][m] * a[m][q];
          a[k][q] = y;
        }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) rowp[tc][4 * p + q] = a[p][q];
    }
    lds_barrier();
    if (tr > jt && tc > jt && (!CHOL || tc <= tr)) {
      double Lt[4][4], Ut[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int k = 0; k < 4; ++k) Lt[p][k] = colp[tr][4 * p + k];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) Ut[k][q] = CHOL ? colp[tc][4 * q + k] : rowp[tc][4 * k + q];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) a[p][q] -= Lt[p][k] * Ut[k][q];
    }
  }
  lds_barrier();
  const int bad = *sbad;
  if (bad < nb) {  // uniform: read after the barrier by every thread
    if (t == 0) info[0] = base + b0 + bad + 1;
    return false;
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 4 * tr + p, c = 4 * tc + q;
      if (r < nb && c < nb && (!CHOL || c <= r)) A[(size_t)(b0 + r) * n + b0 + c] = a[p][q];
    }
  return true;
}

// Cholesky of the CB x CB diagonal block by the four wavefronts of the
// workgroup (256 threads).  The block arrives in LDS (S: lower triangle,
// identity past nb) and leaves as L in A's lower triangle at (b0, b0).
//
// Wave w holds the rows of the 4-row blocks b = w, w + 4, w + 8, w + 12 of
// the symmetric block as FP64 matrix-core accumulators (v_mfma_f64_16x16x4f64
// layout: register r of lane c + 16 g holds row 16 r + 4 w + g, column
// 16 ch + c of chunk ch).  Step J factorizes block J + 1 with the four rows
// of L^T of block J (V_J) in LDS:
// * every other wave subtracts the rank-4 product of V_J from its rows with
//   four matrix-core products (its coefficients as the A operand, V_J as the
//   B operand; rows of finished blocks take zero coefficients);
// * the owner of block J + 1 (wave (J + 1) & 3) holds that block's rows one
//   column per lane, taken from its accumulators one step earlier; it
//   applies V_J to them on the vector ALU (coefficients by LDS broadcast),
//   reads the 4 x 4 diagonal block by readlane, factorizes it as uniform
//   values and solves the rows into V_{J+1}; its own matrix-core products
//   with V_J wait for the next step, off the chain of pivots;
// * the owner of block J + 2 takes that block's rows out of its
//   accumulators once V_J is applied, for the next step.
// With yin (LDS, the block's entries of a right-hand side v, one per row),
// the forward solve L y = v runs alongside: every wave keeps v less the
// solved blocks' terms one row per lane, the owner solves the block's four
// entries of y as uniform values next to its pivots and passes them with
// V_J, and y goes to ydst at the end.
// One barrier per four columns.  A failed pivot does not branch: the first
// failing index is kept and reported after the loop, and the factor (and y)
// is then not written.  buf: CHOL_BUF doubles; S collects the rows of L^T
// once the block is read.
constexpr int CHOL_BUF = 3 * 4 * CB + 4 * 4 * CB + 3 * 4 + CB;

__device__ __forceinline__ bool chol_diag_rows(int n, int b0, double* __restrict__ A, int32_t* __restrict__ info,
                                               int base, double (*S)[CB + 1], double* __restrict__ buf,
                                               int* __restrict__ sbad, const double* yin = nullptr,
                                               double* __restrict__ ydst = nullptr) {
  const int nb = min(CB, n - b0);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lg = lane >> 4;
  double* ext = buf + 3 * 4 * CB + w * 4 * CB;   // this wave's row extraction
  double* ys = buf + 3 * 4 * CB + 4 * 4 * CB;    // y of V_J's block, slot J % 3
  double* yout = ys + 3 * 4;                     // y of the whole block
  const bool wy = yin != nullptr;
  double bv = wy ? yin[lane] : 0.0;              // v less the solved blocks' terms
  dbl4 acc[4];
#pragma unroll
  for (int ch = 0; ch < 4; ++ch)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * r + 4 * w + lg, k = 16 * ch + li;
      acc[ch][r] = i >= k ? S[i][k] : S[k][i];
    }
  if (threadIdx.x == 0) *sbad = CB;
  int bad = CB;
  lds_barrier();
  // block J's rows (this wave's, q = J >> 2) one column per lane, through
  // LDS (the same wave writes and reads)
  auto take_rows = [&](const int J, double (&r)[4]) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) ext[lg * CB + 16 * ch + li] = acc[ch][J >> 2];
#pragma unroll
    for (int t = 0; t < 4; ++t) r[t] = ext[t * CB + lane];
  };
  // block J's rows, every earlier block applied -> rows of L^T (zero left of
  // the pivot), to buf (for the other waves) and S (for the output)
  auto factor_rows = [&](const int J, const double (&r)[4]) {
    const int j0 = 4 * J;
    double a[4][4], Ld[4][4], rp[4], bj[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int m2 = 0; m2 <= m; ++m2) a[m][m2] = readlane_f64(r[m], j0 + m2);
    if (wy) {
#pragma unroll
      for (int m = 0; m < 4; ++m) bj[m] = readlane_f64(bv, j0 + m);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      double d = a[m][m];
#pragma unroll
      for (int p = 0; p < m; ++p) d = fma(-Ld[m][p], Ld[m][p], d);
      bad = (bad == CB && !(d > 0.0 && isfinite(d))) ? j0 + m : bad;
      // 1 / sqrt(d): hardware estimate and one Newton step
      const double y0 = __builtin_amdgcn_rsq(d);
      const double h = 0.5 * y0, g = d * y0;
      rp[m] = fma(y0, fma(-h, g, 0.5), y0);
      Ld[m][m] = d * rp[m];
#pragma unroll
      for (int m2 = m + 1; m2 < 4; ++m2) {
        double v = a[m2][m];
#pragma unroll
        for (int p = 0; p < m; ++p) v = fma(-Ld[m2][p], Ld[m][p], v);
        Ld[m2][m] = v * rp[m];
      }
    }
    double* out = buf + (J % 3) * 4 * CB;
    double l[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      double v = r[m];
#pragma unroll
      for (int p = 0; p < m; ++p) v = fma(-Ld[m][p], l[p], v);
      l[m] = lane >= j0 + m ? v * rp[m] : 0.0;
      out[m * CB + lane] = l[m];
      S[j0 + m][lane] = l[m];
    }
    if (wy) {
      double yv[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        double v = bj[m];
#pragma unroll
        for (int p = 0; p < m; ++p) v = fma(-Ld[m][p], yv[p], v);
        yv[m] = v * rp[m];
      }
      if (lane < 4) {
        const double ym = lane == 0 ? yv[0] : lane == 1 ? yv[1] : lane == 2 ? yv[2] : yv[3];
        ys[(J % 3) * 4 + lane] = ym;
        yout[j0 + lane] = ym;
      }
    }
  };
  double r[4];
  if (w == 0) {
    take_rows(0, r);
    factor_rows(0, r);
  } else if (w == 1) {
    take_rows(1, r);
  }
  lds_barrier();
  // operands of V_J: this wave's coefficients (A, rows of finished blocks
  // zero) and V_J by chunk (B)
  auto operands = [&](const double* vb, const int J, double& aop, double (&bop)[4]) {
    const double av = vb[lg * CB + 16 * (li >> 2) + 4 * w + (li & 3)];
    aop = w + 4 * (li >> 2) > J ? -av : 0.0;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) bop[ch] = vb[lg * CB + 16 * ch + li];
  };
  auto apply = [&](const double aop, const double (&bop)[4]) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) acc[ch] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[ch], acc[ch], 0, 0, 0);
  };
  // V_J sits in buf slot J % 3 until the end of step J + 1: the owner of
  // step J applies it to its accumulators in step J + 1
#pragma unroll
  for (int J = 0; J < CB / 4 - 1; ++J) {
    const double* vb = buf + (J % 3) * 4 * CB;
    // v less block J's terms
    auto take_y = [&](const double (&lv)[4]) {
#pragma unroll
      for (int k = 0; k < 4; ++k) bv = fma(-lv[k], ys[(J % 3) * 4 + k], bv);
    };
    if (w == ((J + 1) & 3)) {
      // block J + 1: V_J on the vector ALU, then its pivots
      const int R0 = 4 * (J + 1);
      double lv[4], cf[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        lv[k] = vb[k * CB + lane];
#pragma unroll
        for (int t = 0; t < 4; ++t) cf[k][t] = vb[k * CB + R0 + t];
      }
      if (wy) take_y(lv);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int k = 0; k < 4; ++k) r[t] = fma(-cf[k][t], lv[k], r[t]);
      factor_rows(J + 1, r);
    } else if (w + 12 > J) {   // the wave still has rows past block J
      if (wy) {
        double lv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) lv[k] = vb[k * CB + lane];
        take_y(lv);
      }
      if (J >= 1 && w == (J & 3)) {
        double daop, dbop[4];
        operands(buf + ((J - 1) % 3) * 4 * CB, J - 1, daop, dbop);
        apply(daop, dbop);
      }
      double aop, bop[4];
      operands(vb, J, aop, bop);
      apply(aop, bop);
      if (J + 2 < CB / 4 && w == ((J + 2) & 3)) take_rows(J + 2, r);
    }
    lds_barrier();
  }
  if (bad < CB && lane == 0) atomicMin(sbad, bad);
  lds_barrier();
  const int bd = *sbad;
  if (bd < nb) {  // uniform: read after the barrier by every thread
    if (threadIdx.x == 0) info[0] = base + b0 + bd + 1;
    return false;
  }
  // S[j][k] = L[k][j]
  const int k = threadIdx.x >> 2, seg = threadIdx.x & 3;
  if (k < nb) {
    double* dst = A + (size_t)(b0 + k) * n + b0 + 16 * seg;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (16 * seg + c <= k) dst[c] = S[16 * seg + c][k];
  }
  if (wy && threadIdx.x < nb) ydst[threadIdx.x] = yout[threadIdx.x];
  return true;
}

template <bool CHOL>
__global__ void __launch_bounds__(256) k_blk_diag(int n, int b0, double* __restrict__ A, int32_t* __restrict__ info,
                                                  int base, const int32_t* __restrict__ skip,
                                                  double* __restrict__ y = nullptr) {
  if (skip && *skip) return;
  if (info[0] != 0) return;
  if constexpr (CHOL) {
    __shared__ double S[CB][CB + 1];
    __shared__ double buf[CHOL_BUF];
    __shared__ int sbad;
    __shared__ double yl[CB];
    const int nb = min(CB, n - b0);
    const double yv = (y && threadIdx.x < CB) ? y[b0 + min((int)threadIdx.x, nb - 1)] : 0.0;
    stage_tile<256>(S, A + (size_t)b0 * n + b0, n, nb, nb, 1.0);
    if (y && threadIdx.x < CB) yl[threadIdx.x] = (int)threadIdx.x < nb ? yv : 0.0;
    lds_barrier();
    chol_diag_rows(n, b0, A, info, base, S, buf, &sbad, y ? yl : nullptr, y ? y + b0 : nullptr);
  } else {
    __shared__ double work[DIAG_WORK];
    diag_factor<false>(n, b0, A, info, base, work);
  }
}

// Panels: wave task t < rows below: row r solves x U11 = a (LU) or
// x L11^T = a (Cholesky); for LU, tasks past the rows solve L11 y = a for a
// column to the right (unit lower).  Lanes hold the CB entries.
template <bool CHOL>
__global__ void k_blk_panel(int n, int b0, double* __restrict__ A, const int32_t* __restrict__ info,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double T[CB][CB + 1];
  __shared__ double rd[CB];
  if (info[0] != 0) return;
  const int nb = min(CB, n - b0);
  const int rest = n - b0 - nb;
  const int lane = threadIdx.x & 63;
  const int task = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  // the wave's row (or LU column) is loaded with the diagonal block
  double v = 0.0;
  if (task < rest)
    v = lane < nb ? A[(size_t)(b0 + nb + task) * n + b0 + lane] : 0.0;
  else if (!CHOL && task < 2 * rest)
    v = lane < nb ? A[(size_t)(b0 + lane) * n + b0 + nb + (task - rest)] : 0.0;
  stage_tile<256>(T, A + (size_t)b0 * n + b0, n, nb, nb, 1.0);
  __syncthreads();
  for (int j = threadIdx.x; j < CB; j += blockDim.x) rd[j] = 1.0 / T[j][j];
  __syncthreads();
  // substitution along the lanes: the solved entry j is broadcast with
  // readlane (a scalar register), so each step is a short dependent chain
  // of vector ALU operations; the factor entries come from LDS off the chain
  if (task < rest) {
    double* a = A + (size_t)(b0 + nb + task) * n + b0;
    for (int j = 0; j < nb; ++j) {
      const double f = CHOL ? T[lane][j] : T[j][lane];
      const double xj = readlane_f64(v, j) * rd[j];
      v = lane == j ? xj : (lane > j ? fma(-xj, f, v) : v);
    }
    if (lane < nb) a[lane] = v;
  } else if (!CHOL && task < 2 * rest) {
    const int c = b0 + nb + (task - rest);
    for (int j = 0; j < nb; ++j) {
      const double f = T[lane][j];
      const double yj = readlane_f64(v, j);
      v = lane > j ? fma(-f, yj, v) : v;
    }
    if (lane < nb) A[(size_t)(b0 + lane) * n + c] = v;
  }
}

// Trailing update A22 -= L21 U12 (LU) or L21 L21^T (Cholesky, lower tiles).
// With fuse, workgroup (0, 0) -- dispatched first -- updates the next
// diagonal block and then factorizes it (diag_factor, or chol_diag_rows
// with the tile handed over in LDS) while the other workgroups finish the
// trailing update.  y (Cholesky, optional): the fused forward solve; the
// workgroups of the first tile column subtract L21 y_k (y_k = y[b0 ..],
// solved by the previous launch) from their rows of y, and workgroup (0, 0)
// then solves the next block's entries through the new diagonal factor.
template <bool CHOL>
__global__ void __launch_bounds__(256) k_blk_update(int n, int b0, double* __restrict__ A,
                                                    int32_t* __restrict__ info, int fuse, int dbase,
                                                    const int32_t* __restrict__ skip,
                                                    double* __restrict__ y = nullptr) {
  if (skip && *skip) return;
  __shared__ double sm[2][CB][CB + 1];
  __shared__ double yk[CB];
  double (*Ls)[CB + 1] = sm[0];
  double (*Us)[CB + 1] = sm[1];
  if (info[0] != 0) return;
  const int nb = min(CB, n - b0);
  const int base = b0 + nb;
  const int ti = blockIdx.y, tj = blockIdx.x;
  if (CHOL && tj > ti) return;
  const int i0 = base + ti * CB, j0 = base + tj * CB;
  const bool ysolve = CHOL && y && tj == 0;
  // FP64 matrix cores (v_mfma_f64_16x16x4f64): wave w takes the 32 x 32
  // quadrant (w >> 1, w & 1) of the tile as 2 x 2 blocks of 16 x 16, over
  // 16 steps of 4 in k.  Operand lanes: A(i, k) from lane i + 16 k, B(k, j)
  // from lane j + 16 k; result register r of lane j + 16 q holds row
  // q + 4 r of column j.  The staged tiles are zero past nb, so k runs to
  // CB.  The wave's entries of the tile to update are loaded first, with
  // the staging, so the write-back does not wait for memory.
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qr = (w >> 1) * 32, qc = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // a Cholesky diagonal tile has nothing to update above its diagonal
  const bool active = !(CHOL && ti == tj && qc > qr);
  double cv[2][2][4];
  if (active) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + qr + 16 * p + lk + 4 * r, j = j0 + qc + 16 * q + li;
          cv[p][q][r] = A[(size_t)min(i, n - 1) * n + min(j, n - 1)];
        }
  }
  // y loads issued ahead of the tile loads
  double ykv = 0.0, yrow = 0.0;
  if (ysolve) {
    if (threadIdx.x < CB) ykv = y[b0 + min((int)threadIdx.x, nb - 1)];
    yrow = y[min(i0 + (int)(threadIdx.x >> 2), n - 1)];
  }
  if (CHOL)
    stage_tile_pair<256, true>(Ls, A + (size_t)i0 * n + b0, n - i0, nb, Us, A + (size_t)j0 * n + b0, n - j0, nb, n,
                               0.0);
  else
    stage_tile_pair<256, false>(Ls, A + (size_t)i0 * n + b0, n - i0, nb, Us, A + (size_t)b0 * n + j0, nb, n - j0, n,
                                0.0);
  if (ysolve && threadIdx.x < CB) yk[threadIdx.x] = (int)threadIdx.x < nb ? ykv : 0.0;
  __syncthreads();
  // y rows i0 .. i0 + 63 -= L21 y_k: thread (row, quarter of the columns)
  double ynew = 0.0;
  if (ysolve) {
    const int r = threadIdx.x >> 2, c4 = threadIdx.x & 3;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int m = 0; m < 16; m += 2) {
      a0 = fma(Ls[r][16 * c4 + m], yk[16 * c4 + m], a0);
      a1 = fma(Ls[r][16 * c4 + m + 1], yk[16 * c4 + m + 1], a1);
    }
    const double sum = group_sum(a0 + a1, 4);
    ynew = i0 + r < n ? yrow - sum : 0.0;
    if (!(fuse && ti == 0) && c4 == 0 && i0 + r < n) y[i0 + r] = ynew;
  }
  // Cholesky with fuse: tile (0, 0) is the next diagonal block; its updated
  // values go to LDS for the factorization instead of back to A
  const bool dtile = CHOL && fuse && ti == 0 && tj == 0;
  double sv[2][2][4];
  if (active) {
    dbl4 acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[p][q] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < CB; k0 += 4) {
      const double a0 = Ls[qr + li][k0 + lk], a1 = Ls[qr + 16 + li][k0 + lk];
      const double b0v = Us[k0 + lk][qc + li], b1v = Us[k0 + lk][qc + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0v, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1v, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0v, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1v, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + qr + 16 * p + lk + 4 * r, j = j0 + qc + 16 * q + li;
          if (dtile) {
            sv[p][q][r] = (i < n && j < n) ? cv[p][q][r] - acc[p][q][r] : (i == j ? 1.0 : 0.0);
          } else if (i < n && j < n && (!CHOL || j <= i)) {
            A[(size_t)i * n + j] = cv[p][q][r] - acc[p][q][r];
          }
        }
  }
  if constexpr (CHOL) {
    if (dtile) {
      __shared__ int sbad;
      __syncthreads();   // every wave is done with the staged tiles
      if (qc <= qr) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) sm[0][qr + 16 * p + lk + 4 * r][qc + 16 * q + li] = sv[p][q][r];
      }
      if (ysolve && (threadIdx.x & 3) == 0) yk[threadIdx.x >> 2] = ynew;   // the next block's y
      lds_barrier();
      static_assert(CHOL_BUF <= CB * (CB + 1), "pivot-row exchange must fit one tile");
      chol_diag_rows(n, base, A, info, dbase, sm[0], &sm[1][0][0], &sbad, ysolve ? yk : nullptr,
                     ysolve ? y + base : nullptr);
    }
  } else {
    if (fuse && ti == 0 && tj == 0) {
      __syncthreads();   // the updated block is in A; the LDS tiles are free
      static_assert(DIAG_WORK <= CB * (CB + 1), "diagonal work area must fit one tile");
      diag_factor<false>(n, base, A, info, dbase, &sm[0][0][0]);
    }
  }
}

__global__ void k_transpose(int n, const double* __restrict__ A, double* __restrict__ B,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = by + k, c = bx + threadIdx.x;
    if (r < n && c < n) t[k][threadIdx.x] = A[(size_t)r * n + c];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = bx + k, c = by + threadIdx.x;
    if (r < n && c < n) B[(size_t)r * n + c] = t[threadIdx.x][k];
  }
}

// Triangular solves with the dense Cholesky factor, L y = -rhs and
// L^T step = y, spread over one workgroup per two blocks of CB rows.  A
// workgroup publishes its solved entries by a flag (release at agent scope
// after its stores); the workgroups that need them wait for the flag
// (acquire).  A workgroup only waits for workgroups dispatched before it
// (forward: lower indices; backward: v = nwg - 1 - blockIdx.x), so every
// awaited workgroup is already running.  Each wait is bounded: on expiry
// info[0] is set to -1 and the solve continues, so every wave exits.
// flags: int32 [nwg] per direction (its own array for each launch), zero
// before the launch; nwg = ceil(n / (2 CB)).

// One thread polls with relaxed loads (an acquire load would invalidate the
// caches at every poll) and takes one acquire fence once the flag is seen;
// the workgroup barrier that follows the call orders the other threads'
// reads after it.
__device__ __forceinline__ void blk_wait(const int32_t* flag, int32_t* info) {
  unsigned it = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
    // after one expiry anywhere, no further waiting
    if (++it > (1u << 20) || __hip_atomic_load(info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 0) {
      __hip_atomic_store(info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// The workgroup barrier orders every thread's stores before thread 0's
// release store of the flag (one cache write-back per publication).
__device__ __forceinline__ void blk_publish(int32_t* flag) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// dinv: inverses of the factor's diagonal blocks, (kb * 2) * CB * CB
// row-major, zero outside each block's corner.
// Each workgroup (512 threads) solves two blocks of CB rows, 2 CB v ..
// 2 CB v + 2 CB: the products with the other workgroups' solved rows come
// first, one flag per workgroup; its second block then takes the first's
// solution through LDS, without another flag.  Factor entries and the
// inverse blocks' rows are loaded before they are needed (those of the next
// awaited workgroup during the wait for the current one).
__global__ void __launch_bounds__(512) k_chol_fwd(int n, const double* __restrict__ L,
                                                  const double* __restrict__ dinv, const double* __restrict__ rhs,
                                                  double* __restrict__ y, int32_t* __restrict__ flags,
                                                  int32_t* __restrict__ info) {
  if (info[0] > 0) return;
  __shared__ double part[2 * CB][5];
  __shared__ double rv[CB];
  __shared__ double ys[CB];
  const int v = blockIdx.x;
  const int R0 = 2 * CB * v, nr = min(2 * CB, n - R0);
  const int nA = min(CB, nr), nB = nr - nA;
  const int t = threadIdx.x;
  // products with earlier workgroups: thread (row r, slice sl of 32 columns
  // of each earlier 2 CB-column block)
  const int r = t >> 2, sl = t & 3;
  const double* Lrow = L + (size_t)(R0 + min(r, nr - 1)) * n + sl * 32;
  // inverse blocks and the block-B-by-block-A factor entries: thread (row i,
  // segment seg of 8 columns)
  const int i = t >> 3, seg = t & 7;
  double dA[8], dB[8], lBA[8];
  {
    const double* DA = dinv + (size_t)(2 * v * 2) * CB * CB + i * CB + seg * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) dA[q] = DA[q];
    if (nB > 0) {
      const double* DB = dinv + (size_t)((2 * v + 1) * 2) * CB * CB + i * CB + seg * 8;
      const double* LB = L + (size_t)(R0 + CB + min(i, nB - 1)) * n + R0 + seg * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        dB[q] = DB[q];
        lBA[q] = LB[q];
      }
    }
  }
  double a0 = 0.0, a1 = 0.0;
  double lv[32];
  if (v > 0) {
#pragma unroll
    for (int q = 0; q < 32; ++q) lv[q] = Lrow[q];
  }
  for (int k = 0; k < v; ++k) {
    double lc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) lc[q] = lv[q];
    if (k + 1 < v) {
#pragma unroll
      for (int q = 0; q < 32; ++q) lv[q] = Lrow[(k + 1) * 2 * CB + q];
    }
    if (t == 0) blk_wait(flags + k, info);
    __syncthreads();
    if (r < nr) {
      const double* yk = y + k * 2 * CB + sl * 32;
#pragma unroll
      for (int q = 0; q < 32; q += 2) {
        a0 += lc[q] * yk[q];
        a1 += lc[q + 1] * yk[q + 1];
      }
    }
  }
  part[r][sl] = a0 + a1;
  __syncthreads();
  if (t < CB) rv[t] = t < nA ? -rhs[R0 + t] - ((part[t][0] + part[t][1]) + (part[t][2] + part[t][3])) : 0.0;
  __syncthreads();
  // block A: y_A = L_AA^{-1} rv
  {
    double sacc = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sacc += dA[q] * rv[seg * 8 + q];
    sacc = group_sum(sacc, 8);
    if (seg == 0) {
      ys[i] = sacc;
      if (i < nA) y[R0 + i] = sacc;
    }
  }
  __syncthreads();
  if (nB > 0) {
    // block B: rv = -rhs_B - (earlier workgroups) - L_BA y_A
    double sacc = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sacc += lBA[q] * ys[seg * 8 + q];
    sacc = group_sum(sacc, 8);
    if (seg == 0) {
      const int rb = CB + i;
      rv[i] = i < nB ? -rhs[R0 + rb] - ((part[rb][0] + part[rb][1]) + (part[rb][2] + part[rb][3])) - sacc : 0.0;
    }
    __syncthreads();
    double sb = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sb += dB[q] * rv[seg * 8 + q];
    sb = group_sum(sb, 8);
    if (seg == 0 && i < nB) y[R0 + CB + i] = sb;
  }
  blk_publish(flags + v);
}

// L^T x = y with the same two-block workgroups, in reverse order (workgroup
// v = nwg - 1 - blockIdx.x, so every awaited workgroup was dispatched
// earlier): block B (the second) first, then block A with x_B through LDS.
__global__ void __launch_bounds__(512) k_chol_bwd(int n, const double* __restrict__ L,
                                                  const double* __restrict__ dinv, const double* __restrict__ y,
                                                  double* __restrict__ x, int32_t* __restrict__ flags,
                                                  int32_t* __restrict__ info) {
  if (info[0] > 0) return;
  __shared__ double part[4][2 * CB];
  __shared__ double rv[CB];
  __shared__ double xs[CB];
  const int nwg = (n + 2 * CB - 1) / (2 * CB);
  const int v = nwg - 1 - blockIdx.x;
  const int R0 = 2 * CB * v, nr = min(2 * CB, n - R0);
  const int nA = min(CB, nr), nB = nr - nA;
  const int t = threadIdx.x;
  // products with later workgroups' rows: thread (column c of this
  // workgroup, slice sl of 32 rows of each later 2 CB-row block)
  const int c = t & (2 * CB - 1), sl = t >> 7;
  const double* Lcol = L + R0 + min(c, nr - 1);
  // thread (column i of a block, segment seg of 8 rows)
  const int i = t >> 3, seg = t & 7;
  double dA[8], dB[8], lBA[8];
  {
    // (L_AA^{-1})^T: entry (row seg * 8 + q, column i) of the inverse
    const double* DA = dinv + (size_t)(2 * v * 2) * CB * CB + (seg * 8) * CB + i;
#pragma unroll
    for (int q = 0; q < 8; ++q) dA[q] = DA[q * CB];
    if (nB > 0) {
      const double* DB = dinv + (size_t)((2 * v + 1) * 2) * CB * CB + (seg * 8) * CB + i;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        dB[q] = DB[q * CB];
        // L[R0 + CB + seg * 8 + q][R0 + i] (rows past the block clamped,
        // weighted by x_B entries that are zero)
        lBA[q] = L[(size_t)(R0 + CB + min(seg * 8 + q, nB - 1)) * n + R0 + i];
      }
    }
  }
  double a0 = 0.0, a1 = 0.0;
  double lv[32];
  auto load_l = [&](int k) {
#pragma unroll
    for (int q = 0; q < 32; ++q) lv[q] = Lcol[(size_t)min(k * 2 * CB + sl * 32 + q, n - 1) * n];
  };
  if (nwg - 1 > v) load_l(nwg - 1);
  for (int k = nwg - 1; k > v; --k) {
    double lc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) lc[q] = lv[q];
    if (k - 1 > v) load_l(k - 1);
    if (t == 0) blk_wait(flags + k, info);
    __syncthreads();
    const int kr0 = k * 2 * CB + sl * 32;
    if (c < nr) {
#pragma unroll
      for (int q = 0; q < 32; q += 2) {
        if (kr0 + q < n) a0 += lc[q] * x[kr0 + q];
        if (kr0 + q + 1 < n) a1 += lc[q + 1] * x[kr0 + q + 1];
      }
    }
  }
  part[sl][c] = a0 + a1;
  __syncthreads();
  if (nB > 0) {
    if (t < CB) {
      const int cb = CB + t;
      rv[t] = t < nB ? y[R0 + cb] - ((part[0][cb] + part[1][cb]) + (part[2][cb] + part[3][cb])) : 0.0;
    }
    __syncthreads();
    // x_B = L_BB^{-T} rv
    double sb = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sb += dB[q] * rv[seg * 8 + q];
    sb = group_sum(sb, 8);
    if (seg == 0) {
      xs[i] = i < nB ? sb : 0.0;
      if (i < nB) x[R0 + CB + i] = sb;
    }
    __syncthreads();
  }
  // block A: rv = y_A - (later workgroups) - L_BA^T x_B
  {
    double sacc = 0.0;
    if (nB > 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) sacc += lBA[q] * xs[seg * 8 + q];
    }
    sacc = group_sum(sacc, 8);
    if (seg == 0)
      rv[i] = i < nA ? y[R0 + i] - ((part[0][i] + part[1][i]) + (part[2][i] + part[3][i])) - sacc : 0.0;
  }
  __syncthreads();
  {
    double sa = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sa += dA[q] * rv[seg * 8 + q];
    sa = group_sum(sa, 8);
    if (seg == 0 && i < nA) x[R0 + i] = sa;
  }
  blk_publish(flags + v);
}

}  // namespace dev
}  // namespace rpf
