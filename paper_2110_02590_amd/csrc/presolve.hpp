// Host presolve of the reduced-space method: everything that depends only on
// the grid topology is computed once here (the paper factorizes the
// Jacobian's static sparsity pattern during presolve and only refactorizes
// numerically afterwards, Section V-A.1).
//
//  * control / state split and equation rows (Section II-B, eq. statecontrol);
//  * a fill-reducing ordering of the state variables (bus-level minimum
//    degree, each bus expanded to theta then v) with static diagonal pivots
//    P_i <-> theta_i, Q_i <-> v_i;
//  * the symbolic LU pattern of J_x in that order (structurally symmetric,
//    so the pattern of L is that of a Cholesky factor and U = L^T), its level
//    sets for forward/backward substitution and the refactorization program;
//  * gather lists that turn per-branch records into J_x, J_u, g, the
//    rank-one constraint gradients and the Lagrangian Hessian K.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace rpf {

enum BusType : int32_t { BUS_PQ = 0, BUS_PV = 1, BUS_REF = 2 };

struct GridData {
  int32_t nb = 0, nl = 0, ng = 0;
  double base_mva = 100.0;
  std::vector<int32_t> bus_type, br_from, br_to, gen_bus;
  std::vector<double> br_r, br_x, br_b, c2, c1, c0;
};

// Branch record layout (one per branch, RECW doubles):
//   [0..3]   P_f, Q_f, P_t, Q_t
//   [4..19]  d(E_e)/d(local k), E_e in (P_f, Q_f, P_t, Q_t), local k in
//            (theta_f, theta_t, v_f, v_t): index 4 + 4*eq + k.
constexpr int RECW = 20;
// Branch second-order record: 4x4 symmetric W (row-major, 16 doubles) and
// the local gradient (4 doubles).
constexpr int WREC = 20;
// leading dimension of the dense tail blocks (and the largest tail)
constexpr int TAIL_MAX = 128;

struct Levels {
  std::vector<int32_t> ptr;   // [nlev + 1]
  std::vector<int32_t> rows;  // rows in schedule order
  int nlev() const { return (int)ptr.size() - 1; }
};

struct Presolve {
  int nb = 0, nl = 0, ng = 0, npv = 0, npq = 0, nx = 0, nu = 0, m = 0, nvar = 0;
  int ref = -1;
  double base_mva = 100.0;
  std::vector<int32_t> pv, pq;          // ascending bus ids
  std::vector<int32_t> gen_at;          // bus -> generator index or -1
  // variables: ids in [0, nvar): internal state order [0, nx), controls
  // [nx, nx + nu) in the paper's order (v_ref, v_pv, p_pv)
  std::vector<int32_t> th_var, v_var;   // per bus, -1 when not a variable
  std::vector<int32_t> p_var;           // per bus (PV only), else -1
  std::vector<int32_t> rowP, rowQ;      // per bus, internal row or -1
  std::vector<int32_t> x_int2paper;     // internal state index -> paper index
  std::vector<int32_t> var_bus;         // per internal state var: bus id
  std::vector<int32_t> var_isv;         // per internal state var: 1 if v, 0 if theta

  // branch local variable ids (theta_f, theta_t, v_f, v_t), -1 if none
  std::vector<int32_t> br_var;          // [nl * 4]
  // bus -> incident branch ends: entries 2*l + e (e = 0 from, 1 to)
  std::vector<int32_t> inc_ptr, inc_end;

  // LU of J_x (internal order), CSR with sorted columns, diagonal position
  std::vector<int32_t> lu_ptr, lu_col, lu_diag;
  // transposed factor (CSR of (L+U)^T) and source positions in lu
  std::vector<int32_t> lut_ptr, lut_col, lut_diag, lut_src;
  // subtree partition: packs [pack_ptr[q], pack_ptr[q+1]) of independent
  // subtrees, then the top rows [t0, nx)
  int subtree_max = 1024;
  int t0 = 0, ntop = 0;
  std::vector<int32_t> pack_ptr;
  std::vector<int32_t> lo_split;   // first lower entry with col >= t0
  std::vector<int32_t> up_split;   // first upper entry with col >= t0
  // pack-local level lists: pack q's forward levels are
  // pk_frows[pk_flev[pk_flev_off[q] + k] .. pk_flev[pk_flev_off[q] + k + 1])
  std::vector<int32_t> pk_flev, pk_flev_off, pk_frows;
  std::vector<int32_t> pk_blev, pk_blev_off, pk_brows;
  // staged programs of the pack solves: for pack rows i < t0, the
  // pack-internal lower (forward) / upper (backward) entries of row i are
  // pkf_pos/pkf_col[pkf_rp[i] .. pkf_rp[i+1]) (LU positions, pack-local
  // columns), likewise pkb_*
  std::vector<int32_t> pkf_rp, pkf_pos, pkb_rp, pkb_pos;
  std::vector<int16_t> pkf_col, pkb_col;
  // dense tails of the packs for the batched solves.  In pack q the rows
  // whose forward level (height in the elimination tree) is at least the
  // pack's cut form an ancestor-closed set T_q of at most tail_max rows
  // (the chains near the subtree roots): ptl_rows[ptl_off[q] ..
  // ptl_off[q+1]) (pack-local, ascending).  The entries of the LU pattern
  // inside T_q x T_q are ptl_pos (LU positions) with dense offsets ptl_dense
  // (a * TAIL_MAX + b, a = row, b = column index within T_q), pack q's from
  // ptl_eoff[q].  The batched programs (levels, rows, staged entries, as
  // pk_*): forward = the other rows by level, then one level of the T rows
  // with only their entries outside T_q; backward = the other rows by level
  // (the T rows are solved before them with the dense inverse).
  int tail_max = 128;
  std::vector<int32_t> ptl_off, ptl_eoff, ptl_pos, ptl_dense;
  std::vector<int16_t> ptl_rows;
  std::vector<int32_t> ptf_lev, ptf_lev_off, ptf_rows, ptb_lev, ptb_lev_off, ptb_rows;
  std::vector<int32_t> ptf_rp, ptf_pos, ptb_rp, ptb_pos;
  std::vector<int16_t> ptf_col, ptb_col;
  // refactorization of the tails, right-looking: for the b-th tail row k of
  // pack q (global tail index ptl_off[q] + b), the LU positions of the L
  // entries (i, k) of the tail rows i > k are rft_pos[rft_ptr[g] ..
  // rft_ptr[g + 1])
  std::vector<int32_t> rft_ptr, rft_pos;
  // top-part levels (global row ids)
  std::vector<int32_t> top_flev, top_frows, top_blev, top_brows;
  // dense top block: LU positions and their dense (row-major) offsets
  std::vector<int32_t> top_pos;
  std::vector<int64_t> top_dense;
  Levels lev_lo;   // forward schedule: L solve, U^T solve, refactor
  Levels lev_up;   // backward schedule: U solve, L^T solve
  // refactorization program: for each L entry p of row i (column k), the
  // target positions in row i of U-row k entries beyond the diagonal
  std::vector<int64_t> upd_ptr;  // [nnz_lu + 1], only L entries non-empty
  std::vector<int32_t> upd_tgt;
  std::vector<int32_t> rf_ustart;  // [nnz_lu], L entries: first U position of the pivot row
  int max_lu_row = 0;

  // gather lists.  Every J_x pattern position (including fill) is a slot;
  // slot sources index branch records (l * RECW + 4 + 4*eq + k).
  std::vector<int32_t> jx_src_ptr, jx_src;       // [nnz_lu + 1]
  // J_u in CSR over internal rows, and its transpose (CSR over controls)
  std::vector<int32_t> ju_ptr, ju_col, ju_src_ptr, ju_src;
  std::vector<double> ju_const;                  // constant part (-1 for p_pv)
  std::vector<int32_t> jut_ptr, jut_col, jut_srcpos;
  // residual rows: sources are record values (l * RECW + eq)
  std::vector<int32_t> g_src_ptr, g_src;
  std::vector<int32_t> row_bus, row_isq, row_pvar;   // per internal row
  // bus injections P_i, Q_i: per bus lists of record value indices
  // (reuse inc lists).
  // rank-one constraint gradients G (rows: p_ref, q_ref, q_pv ascending)
  int nr1 = 0;
  std::vector<int32_t> r1_bus, r1_isq;
  std::vector<int32_t> G_ptr, G_col, G_src_ptr, G_src;
  std::vector<int32_t> Gt_ptr, Gt_col, Gt_srcpos;
  // Lagrangian Hessian K over all variables (CSR, sorted columns); sources
  // index branch second-order records (l * WREC + 4*k1 + k2)
  std::vector<int32_t> K_ptr, K_col, K_src_ptr, K_src, K_diag;
  // local gradient gather: per variable, sources l * WREC + 16 + k
  std::vector<int32_t> vg_src_ptr, vg_src;

  // constraint order: h_f[nl], h_t[nl], v_pq[npq], p_ref, q_ref, q_pv[npv]
  int c_vpq() const { return 2 * nl; }
  int c_pref() const { return 2 * nl + npq; }
  int c_qref() const { return 2 * nl + npq + 1; }
  int c_qpv() const { return 2 * nl + npq + 2; }
};

// Throws std::runtime_error with a message on invalid input.
// subtree_max bounds the rows of one pack of independent subtrees.
Presolve build_presolve(const GridData& g, int subtree_max = 1024, int tail_max = 128);

struct PresolveStats {
  int64_t nnz_jx, nnz_lu, nlev_lo, nlev_up, max_lu_row, refactor_updates, nnz_ju, nnz_k, nnz_g;
  int64_t npacks, ntop, max_pack_levels, top_levels;
  int64_t max_tail_fwd_levels, max_tail_bwd_levels, tail_rows;   // batched programs with dense tails
};
PresolveStats stats(const Presolve& p);

}  // namespace rpf
