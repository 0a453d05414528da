// C ABI of the reduced-space hot path: device buffers owned by the handle,
// launch sequences for the power flow, AL value, reduced gradient, batched
// reduced Hessian-vector products and the dense Cholesky step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <exception>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rpf.h"
#include "kernels.hpp"
#include "qp.hpp"
#include "presolve.hpp"

using namespace rpf;
using namespace rpf::dev;

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw HipError(std::string(#call) + ": " + hipGetErrorString(e_));              \
  } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// Lanes per row (log2) of each level of a single right-hand side pack
// program (levels lev[l] .. lev[l + 1] of rows, entries rp[i] .. rp[i + 1]
// of row i): enough for two entries per lane on the level's longest row,
// at most 64 lanes per row and 256 lanes per level; + 8 when a row of the
// level still has more than two entries per lane.
std::vector<int8_t> level_lanes(const std::vector<int32_t>& lev, const std::vector<int32_t>& rows,
                                const std::vector<int32_t>& rp) {
  const int nl = std::max((int)lev.size() - 1, 0);
  std::vector<int8_t> lg(nl, 0);
  for (int l = 0; l < nl; ++l) {
    const int nrow = lev[l + 1] - lev[l];
    int len = 0;
    for (int k = lev[l]; k < lev[l + 1]; ++k) len = std::max(len, rp[rows[k] + 1] - rp[rows[k]]);
    int g = 0;
    while (g < 6 && (2 << g) < len && (nrow << (g + 1)) <= 256) ++g;
    lg[l] = (int8_t)(g | ((2 << g) < len ? 8 : 0));
  }
  return lg;
}

}  // namespace

struct rpf_grid {
  Presolve P;
  GridData G;
  int max_batch = 0;
  int nr1 = 0;
  std::vector<void*> allocs;
  bool have_point = false;
  double rho = 0.0;

  // ------------------------------------------------------- device topology
  int32_t *th_var, *v_var, *rowP, *rowQ, *x_i2p, *bus_pvpos;
  int32_t *br_f, *br_t;
  double *br_r, *br_x, *br_b;
  int32_t *pb_ptr, *pb_src, *qb_src;
  int32_t *lu_ptr, *lu_col, *lu_diag, *lut_src;
  int32_t *lo_ptr, *lo_rows, *up_ptr, *up_rows;
  int64_t* upd_ptr;
  int32_t* upd_tgt;
  int32_t* rf_ustart;
  int32_t *jx_sp, *jx_s;
  int32_t *ju_ptr, *ju_col, *ju_sp, *ju_s, *jut_ptr, *jut_col, *jut_pos;
  double* ju_const;
  int32_t *g_sp, *g_s, *row_bus, *row_isq, *row_pvar;
  int32_t *G_ptr, *G_col, *G_sp, *G_s, *Gt_ptr, *Gt_col, *Gt_pos;
  int32_t *K_ptr, *K_col, *K_sp, *K_s, *K_diag, *vg_sp, *vg_s;
  int32_t *pq, *pv, *gen_pidx, *pv_gen, *var_kind, *var_aux;
  int32_t *pack_ptr, *lo_split, *up_split, *pk_flev, *pk_flev_off, *pk_frows, *pk_blev, *pk_blev_off, *pk_brows;
  int32_t* topmul_rows = nullptr;   // pack rows with U entries in top columns
  int32_t* tm_off = nullptr;        // per pack: its range of topmul_rows
  int n_topmul_rows = 0;
  int32_t *top_flev, *top_frows, *top_blev, *top_brows, *top_pos;
  int64_t* top_dense;
  double *dense_top, *dense_topT;
  double *top_dinv, *top_dinvT;   // inverse diagonal blocks of the dense top factor
  // dense inverse S^-1 of the top block and its transpose, computed once per
  // point (after the adjoint solve) for the Hessian-vector products
  double *top_inv, *top_invT;
  bool top_inv_ok = false;
  int npacks = 0, max_pack = 0, tw = 16;
  int32_t *pkf_rp, *pkf_pos, *pkb_rp, *pkb_pos;
  int8_t *pk_flg = nullptr, *pk_blg = nullptr;
  int16_t *pkf_col, *pkb_col;
  int tw_top = 8;
  size_t lds_packg = 0;   // LDS of the global-memory batched pack solves
  size_t lds_rf = 0;      // LDS of the LDS-resident pack refactorization (0: not used)
  bool rf_recs_lds = true;   // its row records staged in LDS as well
  int tw_packt = 0;       // column tile of the LDS-tile batched pack solves (0: not used)
  bool sv_packt = false;  // factor values staged in LDS too
  int packt_threads = 1024;   // threads per workgroup of the LDS-tile pack solves
  size_t lds_packt = 0;
  // factor values in the batched programs' order: forward / backward, J_x / J_x^T
  double *pkfv = nullptr, *pkbv = nullptr, *pkfvT = nullptr, *pkbvT = nullptr;
  // batched programs with dense pack tails (Presolve::ptf_* / ptb_* / ptl_*),
  // the tail blocks and their inverses [4][npacks][TAIL_MAX^2] (L_TT^-1,
  // U_TT^-1 and their transposes)
  int32_t *ptf_lev, *ptf_lev_off, *ptf_rows, *ptf_rp, *ptf_pos, *ptb_lev, *ptb_lev_off, *ptb_rows, *ptb_rp,
      *ptb_pos;
  int16_t *ptf_col, *ptb_col, *ptl_rows;
  int32_t *ptl_off, *ptl_eoff, *ptl_pos, *ptl_dense, *rft_ptr, *rft_pos;
  int4 *rf_rowrec = nullptr, *rf_ent = nullptr, *rf_tlrec = nullptr;   // k_rf_pack_lds records
  int32_t* rf_entu0 = nullptr;
  double *tailA = nullptr, *tailM = nullptr;
  size_t lds_limit = 65536, lds_pack_s = 0, lds_pack1 = 0;
  double *c2, *c1, *c0;
  // predication word for the Hessian-product batches (set while the bounded
  // QP assembles its Schur complements; null otherwise)
  const int32_t* skipw = nullptr;
  // bounded-QP workspace: [n] vectors (n = n_u + m), [m], [n_u], scalars,
  // partial sums of the transposed products
  double *qg, *qd_, *qtl, *qtu, *qzl, *qzu, *qsig, *qbase, *qdda, *qdzla, *qdzua, *qrhs, *qdd, *qdzl, *qdzu;
  double *qcs, *qgn, *qts, *qJv, *qrneg, *qxu, *qHd, *qJt, *qscal, *qpart;
  double* s_try = nullptr;
  double* qS = nullptr;   // the Schur complement before regularisation [n_u x n_u]
  int32_t* qflags = nullptr;
  int qparts = 64;

  // ------------------------------------------------------------ workspace
  double *xi, *th, *vm, *rec, *g, *partial, *resid_d, *d;
  double *luv, *lutv, *juv, *Gv, *Kv, *wrec, *kappa, *a, *b, *Pbus, *Qbus;
  double *cvec, *wvec, *terms, *varg, *lam;
  double *D, *Y, *T, *chol_work;
  // the batches of rpf_reduced_hessian run on nhs internal streams, each
  // with its own D, Y, T workspace (slot 0 is D, Y, T above)
  static constexpr int HS = 8;
  int nhs = 1;
  hipStream_t hs[HS] = {};
  hipEvent_t ev_fork = nullptr, ev_join[HS] = {};
  double *Dk[HS] = {}, *Yk[HS] = {}, *Tk[HS] = {};
  int32_t* chol_flags;   // block flags of the dense triangular solves [2 cdiv(n_u, CB)]
  double* chol_dinv;     // inverses of the Cholesky factor's diagonal blocks
  // tracking step workspace
  double *Hbuf, *Kbuf, *gradbuf, *dstep, *u_try, *xi_save, *scur, *pdt, *qdt, *tres;
  int32_t* tflags;
  int32_t *flag, *piv_status;
  double* rdiag;   // 1 / u_ii of the refactorized rows [n_x]

  int rf_waves = 16;

  // event timing per kernel class
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (class, index of start event)

  size_t prof_begin(hipStream_t s) {
    if (ev_used + 2 > ev_pool.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ev_pool.push_back(e);
      }
    }
    size_t i = ev_used;
    ev_used += 2;
    HIPCHK(hipEventRecord(ev_pool[i], s));
    return i;
  }
  void prof_end(int cls, size_t i, hipStream_t s) {
    HIPCHK(hipEventRecord(ev_pool[i + 1], s));
    ev_marks.push_back({cls, i});
  }

  // per-call device timings, when RPF_TRACE was set (not empty, not "0")
  // as the handle was created: two events around each traced call, each
  // call reported as one JSON line on stderr once both have completed
  // (polled at later calls, waited for when the handle is destroyed)
  struct TraceRec {
    const char* name;
    hipEvent_t a, b;
    long long arg;
  };
  bool trace_on = false;
  std::deque<TraceRec> trace_q;
  std::vector<hipEvent_t> trace_free;
  hipEvent_t trace_event() {
    if (trace_free.empty()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = trace_free.back();
    trace_free.pop_back();
    return e;
  }
  void trace_report(bool wait) {
    while (!trace_q.empty()) {
      TraceRec r = trace_q.front();
      if (wait) {
        if (hipEventSynchronize(r.b) != hipSuccess) (void)hipGetLastError();
      } else if (hipEventQuery(r.b) != hipSuccess) {
        (void)hipGetLastError();   // not ready: not an error of the next call
        break;
      }
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess)
        std::fprintf(stderr, "{\"rpf_trace\": \"%s\", \"ms\": %.4f, \"arg\": %lld}\n", r.name, ms, r.arg);
      else
        (void)hipGetLastError();
      trace_free.push_back(r.a);
      trace_free.push_back(r.b);
      trace_q.pop_front();
    }
  }

  template <class T>
  T* up(const std::vector<T>& v) {
    size_t n = std::max<size_t>(v.size(), 1);
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    allocs.push_back(p);
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return (T*)p;
  }
  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    allocs.push_back(p);
    HIPCHK(hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(T)));
    return (T*)p;
  }
  ~rpf_grid() {
    if (trace_on) trace_report(true);
    for (hipEvent_t e : trace_free) (void)hipEventDestroy(e);
    for (int k = 0; k < HS; ++k) {
      if (hs[k]) (void)hipStreamDestroy(hs[k]);
      if (ev_join[k]) (void)hipEventDestroy(ev_join[k]);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
  }
};

// Traced call (see rpf_grid::trace_on); calls on a stream that is capturing
// a graph are not traced, and a call that fails reports nothing.
struct Traced {
  rpf_grid* h;
  const char* name;
  hipStream_t s;
  long long arg;
  hipEvent_t a = nullptr;
  Traced(rpf_grid* h_, const char* name_, hipStream_t s_, long long arg_ = 0)
      : h(h_), name(name_), s(s_), arg(arg_) {
    if (!h->trace_on) return;
    h->trace_report(false);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
      (void)hipGetLastError();
      return;
    }
    a = h->trace_event();
    HIPCHK(hipEventRecord(a, s));
  }
  ~Traced() {
    if (!a) return;
    if (std::uncaught_exceptions() > 0) {
      h->trace_free.push_back(a);
      return;
    }
    hipEvent_t b = nullptr;
    if (!h->trace_free.empty()) {
      b = h->trace_free.back();
      h->trace_free.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
      b = nullptr;
    }
    if (!b || hipEventRecord(b, s) != hipSuccess) {
      (void)hipGetLastError();
      h->trace_free.push_back(a);
      if (b) h->trace_free.push_back(b);
      return;
    }
    h->trace_q.push_back({name, a, b, arg});
  }
  Traced(const Traced&) = delete;
  Traced& operator=(const Traced&) = delete;
};

namespace {

void setup(rpf_grid* h) {
  const Presolve& P = h->P;
  const GridData& G = h->G;
  h->nr1 = P.nr1;
  std::vector<int32_t> bus_pvpos(P.nb, -1);
  for (int k = 0; k < P.npv; ++k) bus_pvpos[P.pv[k]] = k;
  h->th_var = h->up(P.th_var);
  h->v_var = h->up(P.v_var);
  h->rowP = h->up(P.rowP);
  h->rowQ = h->up(P.rowQ);
  h->x_i2p = h->up(P.x_int2paper);
  h->bus_pvpos = h->up(bus_pvpos);
  h->br_f = h->up(G.br_from);
  h->br_t = h->up(G.br_to);
  h->br_r = h->up(G.br_r);
  h->br_x = h->up(G.br_x);
  h->br_b = h->up(G.br_b);
  // bus injection gather lists
  std::vector<int32_t> pbs, qbs;
  for (int i = 0; i < P.nb; ++i)
    for (int q = P.inc_ptr[i]; q < P.inc_ptr[i + 1]; ++q) {
      int l = P.inc_end[q] >> 1, e = P.inc_end[q] & 1;
      pbs.push_back(l * RECW + 2 * e);
      qbs.push_back(l * RECW + 2 * e + 1);
    }
  h->pb_ptr = h->up(P.inc_ptr);
  h->pb_src = h->up(pbs);
  h->qb_src = h->up(qbs);
  h->lu_ptr = h->up(P.lu_ptr);
  h->lu_col = h->up(P.lu_col);
  h->lu_diag = h->up(P.lu_diag);
  h->lut_src = h->up(P.lut_src);
  h->lo_ptr = h->up(P.lev_lo.ptr);
  h->lo_rows = h->up(P.lev_lo.rows);
  h->up_ptr = h->up(P.lev_up.ptr);
  h->up_rows = h->up(P.lev_up.rows);
  h->upd_ptr = h->up(P.upd_ptr);
  {
    // padded by 64 entries: the refactorization loads targets unconditionally
    std::vector<int32_t> tg(P.upd_tgt);
    tg.resize(tg.size() + 64, 0);
    h->upd_tgt = h->up(tg);
  }
  h->rf_ustart = h->up(P.rf_ustart);
  h->jx_sp = h->up(P.jx_src_ptr);
  h->jx_s = h->up(P.jx_src);
  h->ju_ptr = h->up(P.ju_ptr);
  h->ju_col = h->up(P.ju_col);
  h->ju_sp = h->up(P.ju_src_ptr);
  h->ju_s = h->up(P.ju_src);
  h->ju_const = h->up(P.ju_const);
  h->jut_ptr = h->up(P.jut_ptr);
  h->jut_col = h->up(P.jut_col);
  h->jut_pos = h->up(P.jut_srcpos);
  h->g_sp = h->up(P.g_src_ptr);
  h->g_s = h->up(P.g_src);
  h->row_bus = h->up(P.row_bus);
  h->row_isq = h->up(P.row_isq);
  h->row_pvar = h->up(P.row_pvar);
  h->G_ptr = h->up(P.G_ptr);
  h->G_col = h->up(P.G_col);
  h->G_sp = h->up(P.G_src_ptr);
  h->G_s = h->up(P.G_src);
  h->Gt_ptr = h->up(P.Gt_ptr);
  h->Gt_col = h->up(P.Gt_col);
  h->Gt_pos = h->up(P.Gt_srcpos);
  h->K_ptr = h->up(P.K_ptr);
  h->K_col = h->up(P.K_col);
  h->K_sp = h->up(P.K_src_ptr);
  h->K_s = h->up(P.K_src);
  h->K_diag = h->up(P.K_diag);
  h->vg_sp = h->up(P.vg_src_ptr);
  h->vg_s = h->up(P.vg_src);
  h->pq = h->up(P.pq);
  h->pv = h->up(P.pv);
  std::vector<int32_t> gen_pidx(P.ng, -1), pv_gen(P.npv, 0);
  for (int k = 0; k < P.npv; ++k) {
    int gi = P.gen_at[P.pv[k]];
    gen_pidx[gi] = 1 + P.npv + k;
    pv_gen[k] = gi;
  }
  h->gen_pidx = h->up(gen_pidx);
  h->pv_gen = h->up(pv_gen);
  std::vector<int32_t> kind(P.nvar, 0), aux(P.nvar, -1);
  for (int c = 0; c < P.nx; ++c)
    if (P.var_isv[c]) {
      kind[c] = 1;
      int bus = P.var_bus[c];
      aux[c] = (int)(std::lower_bound(P.pq.begin(), P.pq.end(), bus) - P.pq.begin());
    }
  kind[P.nx] = 2;
  for (int k = 0; k < P.npv; ++k) {
    kind[P.nx + 1 + k] = 2;
    kind[P.nx + 1 + P.npv + k] = 3;
    aux[P.nx + 1 + P.npv + k] = k;
  }
  h->var_kind = h->up(kind);
  h->var_aux = h->up(aux);
  h->c2 = h->up(G.c2);
  h->c1 = h->up(G.c1);
  h->c0 = h->up(G.c0);
  h->pack_ptr = h->up(P.pack_ptr);
  h->lo_split = h->up(P.lo_split);
  h->up_split = h->up(P.up_split);
  {
    std::vector<int32_t> rows;
    for (int i = 0; i < P.t0; ++i)
      if (P.up_split[i] < P.lu_ptr[i + 1]) rows.push_back(i);
    h->n_topmul_rows = (int)rows.size();
    h->topmul_rows = h->up(rows);
    // per pack: its rows' range in that ascending list
    const int npk = (int)P.pack_ptr.size() - 1;
    std::vector<int32_t> off(npk + 1, 0);
    for (int q = 0; q < npk; ++q)
      off[q + 1] = (int)(std::lower_bound(rows.begin(), rows.end(), P.pack_ptr[q + 1]) - rows.begin());
    h->tm_off = h->up(off);
  }
  h->pk_flev = h->up(P.pk_flev);
  h->pk_flev_off = h->up(P.pk_flev_off);
  h->pk_frows = h->up(P.pk_frows);
  h->pk_blev = h->up(P.pk_blev);
  h->pk_blev_off = h->up(P.pk_blev_off);
  h->pk_flg = h->up(level_lanes(P.pk_flev, P.pk_frows, P.pkf_rp));
  h->pk_blg = h->up(level_lanes(P.pk_blev, P.pk_brows, P.pkb_rp));
  h->pk_brows = h->up(P.pk_brows);
  h->top_flev = h->up(P.top_flev);
  h->top_frows = h->up(P.top_frows);
  h->top_blev = h->up(P.top_blev);
  h->top_brows = h->up(P.top_brows);
  h->top_pos = h->up(P.top_pos);
  h->top_dense = h->up(P.top_dense);
  h->pkf_rp = h->up(P.pkf_rp);
  h->pkf_pos = h->up(P.pkf_pos);
  h->pkf_col = h->up(P.pkf_col);
  h->pkb_rp = h->up(P.pkb_rp);
  h->pkb_pos = h->up(P.pkb_pos);
  h->pkb_col = h->up(P.pkb_col);
  h->ptf_lev = h->up(P.ptf_lev);
  h->ptf_lev_off = h->up(P.ptf_lev_off);
  h->ptf_rows = h->up(P.ptf_rows);
  h->ptf_rp = h->up(P.ptf_rp);
  h->ptf_pos = h->up(P.ptf_pos);
  h->ptf_col = h->up(P.ptf_col);
  h->ptb_lev = h->up(P.ptb_lev);
  h->ptb_lev_off = h->up(P.ptb_lev_off);
  h->ptb_rows = h->up(P.ptb_rows);
  h->ptb_rp = h->up(P.ptb_rp);
  h->ptb_pos = h->up(P.ptb_pos);
  h->ptb_col = h->up(P.ptb_col);
  h->ptl_off = h->up(P.ptl_off);
  h->ptl_rows = h->up(P.ptl_rows);
  h->ptl_eoff = h->up(P.ptl_eoff);
  h->ptl_pos = h->up(P.ptl_pos);
  h->ptl_dense = h->up(P.ptl_dense);
  h->rft_ptr = h->up(P.rft_ptr);
  h->rft_pos = h->up(P.rft_pos);
  {
    // records of the LDS-resident pack refactorization (k_rf_pack_lds):
    // per program position, per elimination-list entry, per tail entry
    auto i4 = [](std::vector<int32_t>& v) {
      std::vector<int4> r(v.size() / 4);
      std::memcpy(r.data(), v.data(), v.size() * sizeof(int32_t));
      return r;
    };
    auto u32 = [&](int64_t u) {
      if (u > INT32_MAX) throw std::runtime_error("refactorization updates exceed 2^31");
      return (int32_t)u;
    };
    std::vector<int32_t> rr, en, eu, tl;
    for (size_t r = 0; r < P.ptf_rows.size(); ++r) {
      const int i = P.ptf_rows[r];
      rr.insert(rr.end(), {i, P.lu_diag[i], P.ptf_rp[i], P.ptf_rp[i + 1]});
    }
    for (size_t e = 0; e < P.ptf_pos.size(); ++e) {
      const int q = P.ptf_pos[e];
      en.insert(en.end(), {q, P.lu_col[q], P.rf_ustart[q], u32(P.upd_ptr[q + 1] - P.upd_ptr[q])});
      eu.push_back(u32(P.upd_ptr[q]));
    }
    for (size_t c = 0; c < P.rft_pos.size(); ++c) {
      const int q = P.rft_pos[c];
      tl.insert(tl.end(), {q, P.rf_ustart[q], u32(P.upd_ptr[q + 1] - P.upd_ptr[q]), u32(P.upd_ptr[q])});
    }
    // the kernel finds tail pivot b as the b-th row of its pack's last
    // forward level
    const int npk = (int)P.pack_ptr.size() - 1;
    for (int q = 0; q < npk; ++q) {
      const int nT = P.ptl_off[q + 1] - P.ptl_off[q];
      if (nT == 0) continue;
      const int lv = P.ptf_lev_off[q + 1] - 1;
      if (P.ptf_lev[lv + 1] - P.ptf_lev[lv] != nT)
        throw std::runtime_error("internal: the tail rows are not the last forward level");
      for (int b = 0; b < nT; ++b)
        if (P.ptf_rows[P.ptf_lev[lv] + b] != P.pack_ptr[q] + P.ptl_rows[P.ptl_off[q] + b])
          throw std::runtime_error("internal: tail rows out of order in the last forward level");
    }
    // one record past the end of the entry lists: a row with an empty list
    // still reads the record at its (final) start
    en.insert(en.end(), {0, 0, 0, 0});
    eu.push_back(0);
    if (rr.empty()) rr.assign(4, 0);
    if (tl.empty()) tl.assign(4, 0);
    h->rf_rowrec = h->up(i4(rr));
    h->rf_ent = h->up(i4(en));
    h->rf_entu0 = h->up(eu);
    h->rf_tlrec = h->up(i4(tl));
  }
  {
    const size_t npk = P.pack_ptr.size() - 1, blk = (size_t)TAIL_MAX * TAIL_MAX;
    h->tailA = h->alloc<double>(std::max<size_t>(1, npk * 2 * blk));
    h->tailM = h->alloc<double>(std::max<size_t>(1, npk * 4 * blk));
  }
  // padded: the batched pack solves prefetch up to one entry past a pack
  h->pkfv = h->alloc<double>(P.ptf_pos.size() + 64);
  h->pkfvT = h->alloc<double>(P.ptf_pos.size() + 64);
  h->pkbv = h->alloc<double>(P.ptb_pos.size() + 64);
  h->pkbvT = h->alloc<double>(P.ptb_pos.size() + 64);
  h->dense_top = h->alloc<double>((size_t)P.ntop * P.ntop);
  h->dense_topT = h->alloc<double>((size_t)P.ntop * P.ntop);
  h->top_dinv = h->alloc<double>((size_t)cdiv(P.ntop, CB) * 2 * CB * CB);
  h->top_dinvT = h->alloc<double>((size_t)cdiv(P.ntop, CB) * 2 * CB * CB);
  h->top_inv = h->alloc<double>((size_t)P.ntop * P.ntop);
  h->top_invT = h->alloc<double>((size_t)P.ntop * P.ntop);
  h->npacks = (int)P.pack_ptr.size() - 1;
  for (int q = 0; q < h->npacks; ++q) h->max_pack = std::max(h->max_pack, P.pack_ptr[q + 1] - P.pack_ptr[q]);
  {
    int dev = 0, lim = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    h->lds_limit = (size_t)std::max(lim, 32768);
    // single right-hand side pack solves, either direction: LDS of the
    // largest pack with level records (k_pack_solve_1) and without them
    // (k_pack_solve_s, for packs where the records do not fit)
    for (int q = 0; q < h->npacks; ++q) {
      const int r0 = P.pack_ptr[q], nr = P.pack_ptr[q + 1] - r0;
      const int nef = P.pkf_rp[r0 + nr] - P.pkf_rp[r0], neb = P.pkb_rp[r0 + nr] - P.pkb_rp[r0];
      const int nlf = P.pk_flev_off[q + 1] - P.pk_flev_off[q], nlb = P.pk_blev_off[q + 1] - P.pk_blev_off[q];
      h->lds_pack_s = std::max(h->lds_pack_s, pack_lds_bytes(nr, std::max(nef, neb), std::max(nlf, nlb), 1));
      h->lds_pack1 = std::max(h->lds_pack1, pack1_lds_bytes(nr, std::max(nef, neb), std::max(nlf, nlb)));
    }
    // global-memory batched pack solves: largest pack, either direction
    for (int q = 0; q < h->npacks; ++q) {
      const int r0 = P.pack_ptr[q], nr = P.pack_ptr[q + 1] - r0;
      const int seg = P.lu_ptr[r0 + nr] - P.lu_ptr[r0];
      const int nl = std::max(P.pk_flev_off[q + 1] - P.pk_flev_off[q], P.pk_blev_off[q + 1] - P.pk_blev_off[q]);
      h->lds_packg = std::max(h->lds_packg, packg_lds_bytes(nr, seg, nl));
    }
    // LDS-tile batched pack solves: the first variant whose largest pack
    // fits, in the order (8 columns, values staged), (16 columns), (8
    // columns); RPF_PACK_TW = 8 or 16 and RPF_PACK_SV = 0 or 1 pick one
    {
      struct V { int tw; bool sv; };
      std::vector<V> order = {{16, false}, {8, true}, {8, false}};
      if (const char* e = std::getenv("RPF_PACK_TW")) {
        const int tw = std::atoi(e);
        bool sv = tw == 8;
        if (const char* f = std::getenv("RPF_PACK_SV")) sv = std::atoi(f) != 0;
        if (tw == 8 || tw == 16) order.insert(order.begin(), V{tw, sv && tw == 8});
      }
      // the kernel packs a row's first entry and length into one word:
      // entries of a pack below 2^20, row lengths below 2^11
      bool fits_word = true;
      for (int q = 0; q < h->npacks; ++q) {
        const int r0 = P.pack_ptr[q], nr = P.pack_ptr[q + 1] - r0;
        for (const auto* rpv : {&P.ptf_rp, &P.ptb_rp}) {
          if ((*rpv)[r0 + nr] - (*rpv)[r0] >= (1 << 20)) fits_word = false;
          for (int r = r0; r < r0 + nr; ++r)
            if ((*rpv)[r + 1] - (*rpv)[r] >= (1 << 11)) fits_word = false;
        }
      }
      for (const V& v : order) {
        if (!fits_word) break;
        size_t mx = 0;
        for (int q = 0; q < h->npacks; ++q) {
          const int r0 = P.pack_ptr[q], nr = P.pack_ptr[q + 1] - r0;
          const int nef = P.ptf_rp[r0 + nr] - P.ptf_rp[r0], neb = P.ptb_rp[r0 + nr] - P.ptb_rp[r0];
          const int nlf = P.ptf_lev_off[q + 1] - P.ptf_lev_off[q], nlb = P.ptb_lev_off[q + 1] - P.ptb_lev_off[q];
          mx = std::max(mx, packt_lds_bytes(nr, std::max(nef, neb), std::max(nlf, nlb), v.tw, v.sv));
        }
        if (mx <= h->lds_limit) {
          h->tw_packt = v.tw;
          h->sv_packt = v.sv;
          h->lds_packt = mx;
          break;
        }
      }
    }
    // LDS-resident refactorization: values of the pack's CSR rows + pivots
    // + the program's row records
    {
      size_t mx = 0, mxr = 0;
      for (int q = 0; q < h->npacks; ++q) {
        const int r0 = P.pack_ptr[q], nr = P.pack_ptr[q + 1] - r0;
        const int nprog = P.ptf_lev[P.ptf_lev_off[q + 1]] - P.ptf_lev[P.ptf_lev_off[q]];
        const size_t v = (size_t)(P.lu_ptr[r0 + nr] - P.lu_ptr[r0] + nr) * sizeof(double);
        mx = std::max(mx, v);
        mxr = std::max(mxr, v + 16 + (size_t)nprog * sizeof(int4));
      }
      // the row records in LDS too when they fit, else read from memory
      h->rf_recs_lds = mxr <= h->lds_limit;
      h->lds_rf = h->rf_recs_lds ? mxr : (mx <= h->lds_limit ? mx : 0);
    }
    if (h->lds_pack_s > h->lds_limit) throw std::runtime_error("a pack of subtrees does not fit in LDS");
    // the dense top solve also holds two static tiles (about 50 KB)
    const size_t top_static = 52 * 1024;
    h->tw_top = 4;   // 4 columns per workgroup: about one workgroup per CU at 1024 columns
    while (h->tw_top > 1 && (size_t)P.ntop * h->tw_top * 8 + top_static > h->lds_limit) h->tw_top /= 2;
    if ((size_t)P.ntop * 8 + top_static > h->lds_limit)
      throw std::runtime_error("top part of the elimination tree too large for LDS");
    // allow the dynamic LDS sizes above the default for the solve kernels
    const int ldsmax = (int)h->lds_limit;
    auto allow = [&](const void* f) {
      HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, ldsmax));
    };
    auto allow_top = [&](const void* f) {
      HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, ldsmax - (int)top_static));
    };
    allow_top((const void*)k_top_dense);

    if (h->lds_packg > h->lds_limit) throw std::runtime_error("a pack of subtrees does not fit in LDS");
    if (h->lds_rf > 0) allow(h->rf_recs_lds ? (const void*)k_rf_pack_lds<true> : (const void*)k_rf_pack_lds<false>);
#define RPF_ALLOW_PACKT(TW, SV)                                 \
  allow((const void*)k_pack_solve_t<TW, true, true, SV>);       \
  allow((const void*)k_pack_solve_t<TW, true, false, SV>);      \
  allow((const void*)k_pack_solve_t<TW, false, true, SV>);      \
  allow((const void*)k_pack_solve_t<TW, false, false, SV>);
    if (h->tw_packt == 16) { RPF_ALLOW_PACKT(16, false) }
    if (h->tw_packt == 8 && !h->sv_packt) { RPF_ALLOW_PACKT(8, false) }
    if (h->tw_packt == 8 && h->sv_packt) { RPF_ALLOW_PACKT(8, true) }
#undef RPF_ALLOW_PACKT
    allow((const void*)k_pack_solve_g<true, true>);
    allow((const void*)k_pack_solve_g<true, false>);
    allow((const void*)k_pack_solve_g<false, true>);
    allow((const void*)k_pack_solve_g<false, false>);
    allow((const void*)k_pack_solve_s<1, true, true>);
    allow((const void*)k_pack_solve_s<1, true, false>);
    allow((const void*)k_pack_solve_s<1, false, true>);
    allow((const void*)k_pack_solve_s<1, false, false>);
    allow((const void*)k_pack_solve_1<true, true>);
    allow((const void*)k_pack_solve_1<true, false>);
    allow((const void*)k_pack_solve_1<false, true>);
    allow((const void*)k_pack_solve_1<false, false>);
  }
  const size_t nnz = P.lu_col.size();
  h->xi = h->alloc<double>(P.nx);
  h->th = h->alloc<double>(P.nb);
  h->vm = h->alloc<double>(P.nb);
  h->rec = h->alloc<double>((size_t)P.nl * RECW);
  h->g = h->alloc<double>(P.nx);
  h->partial = h->alloc<double>(cdiv(std::max(P.nx, P.m + P.ng), 256) + 8);
  h->resid_d = h->alloc<double>(4);
  h->d = h->alloc<double>(P.nx);
  h->luv = h->alloc<double>(nnz);
  h->lutv = h->alloc<double>(nnz);
  h->juv = h->alloc<double>(P.ju_col.size());
  h->Gv = h->alloc<double>(P.G_col.size());
  h->Kv = h->alloc<double>(P.K_col.size());
  h->wrec = h->alloc<double>((size_t)P.nl * WREC);
  h->kappa = h->alloc<double>(P.nr1);
  h->a = h->alloc<double>(P.nb);
  h->b = h->alloc<double>(P.nb);
  h->Pbus = h->alloc<double>(P.nb);
  h->Qbus = h->alloc<double>(P.nb);
  h->cvec = h->alloc<double>(P.m);
  h->wvec = h->alloc<double>(P.m);
  h->terms = h->alloc<double>(P.m + P.ng);
  h->varg = h->alloc<double>(P.nvar);
  h->lam = h->alloc<double>(P.nx);
  h->D = h->alloc<double>((size_t)P.nvar * h->max_batch);
  h->Y = h->alloc<double>((size_t)P.nvar * h->max_batch);
  h->T = h->alloc<double>((size_t)P.nr1 * h->max_batch);
  h->Dk[0] = h->D;
  h->Yk[0] = h->Y;
  h->Tk[0] = h->T;
  // batches one after the other on the caller's stream (with the dense pack
  // tails, concurrent batches on three streams measured no faster);
  // RPF_HVP_STREAMS = 2 .. 8 runs them on that many handle-owned streams
  h->nhs = 1;
  if (const char* e = std::getenv("RPF_HVP_STREAMS")) h->nhs = std::max(1, std::min(rpf_grid::HS, std::atoi(e)));
  // 512 threads (16-column tiles only): two workgroups per CU when a
  // pack's tile fits twice in LDS
  if (const char* e = std::getenv("RPF_PACK_THREADS"))
    if (std::atoi(e) == 512 && h->tw_packt == 16) h->packt_threads = 512;
  if (h->nhs > 1) {
    HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    for (int k = 0; k < h->nhs; ++k) {
      HIPCHK(hipStreamCreateWithFlags(&h->hs[k], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&h->ev_join[k], hipEventDisableTiming));
      if (k > 0) {
        h->Dk[k] = h->alloc<double>((size_t)P.nvar * h->max_batch);
        h->Yk[k] = h->alloc<double>((size_t)P.nvar * h->max_batch);
        h->Tk[k] = h->alloc<double>((size_t)P.nr1 * h->max_batch);
      }
    }
  }
  h->chol_work = h->alloc<double>(P.nu);
  h->chol_flags = h->alloc<int32_t>(2 * (size_t)cdiv(P.nu, CB));
  h->chol_dinv = h->alloc<double>((size_t)cdiv(P.nu, CB) * 2 * CB * CB);
  h->Hbuf = h->alloc<double>((size_t)P.nu * P.nu);
  h->Kbuf = h->alloc<double>((size_t)P.nu * P.nu);
  h->gradbuf = h->alloc<double>(P.nu);
  h->dstep = h->alloc<double>(P.nu);
  h->u_try = h->alloc<double>(P.nu);
  h->xi_save = h->alloc<double>(P.nx);
  h->scur = h->alloc<double>(P.m);
  h->s_try = h->alloc<double>(P.m);
  h->pdt = h->alloc<double>(P.nb);
  h->qdt = h->alloc<double>(P.nb);
  h->tres = h->alloc<double>(4);
  h->tflags = h->alloc<int32_t>(8);
  h->flag = h->alloc<int32_t>(4);
  h->piv_status = h->alloc<int32_t>(4);
  h->rdiag = h->alloc<double>(P.nx);
  {
    const size_t n = (size_t)P.nu + P.m;
    double** vn[] = {&h->qg, &h->qd_, &h->qtl, &h->qtu, &h->qzl, &h->qzu, &h->qsig, &h->qbase, &h->qdda,
                     &h->qdzla, &h->qdzua, &h->qrhs, &h->qdd, &h->qdzl, &h->qdzu};
    for (double** v : vn) *v = h->alloc<double>(n);
    double** vm[] = {&h->qcs, &h->qgn, &h->qts, &h->qJv};
    for (double** v : vm) *v = h->alloc<double>(P.m);
    double** vu[] = {&h->qrneg, &h->qxu, &h->qHd, &h->qJt};
    for (double** v : vu) *v = h->alloc<double>(P.nu);
    h->qscal = h->alloc<double>(QS_NSCAL);
    h->qparts = std::max(1, std::min(64, cdiv(P.m, 256)));
    h->qpart = h->alloc<double>((size_t)h->qparts * P.nu);
    h->qflags = h->alloc<int32_t>(QF_N);
    h->qS = h->alloc<double>((size_t)P.nu * P.nu);
  }

  int maxrow = std::max(P.max_lu_row, 1);
  int waves = 16;
  while (waves > 1 && (size_t)waves * maxrow * 8 > 65536) waves /= 2;
  if ((size_t)waves * maxrow * 8 > 65536) throw std::runtime_error("LU row too long for LDS staging");
  h->rf_waves = waves;
}

// ---------------------------------------------------------- launch helpers
void state_and_records(rpf_grid* h, const double* u, hipStream_t s, const int32_t* skip = nullptr) {
  const Presolve& P = h->P;
  k_bus_state<<<cdiv(P.nb, 256), 256, 0, s>>>(P.nb, P.nx, h->th_var, h->v_var, h->xi, u, h->th, h->vm, skip);
  LAUNCHCHK();
  k_branch_eval<<<cdiv(P.nl, 256), 256, 0, s>>>(P.nl, h->br_f, h->br_t, h->br_r, h->br_x, h->br_b, h->th,
                                                 h->vm, h->rec, skip);
  LAUNCHCHK();
}

void x_in(rpf_grid* h, const double* x, hipStream_t s, const int32_t* skip = nullptr) {
  k_permute_gather<<<cdiv(h->P.nx, 256), 256, 0, s>>>(h->P.nx, h->x_i2p, x, h->xi, skip);
  LAUNCHCHK();
}

// Blocked dense LU (no pivoting) or Cholesky of a row-major n x n matrix.
// y (Cholesky only, optional): the forward solve L y = v fused into the
// factorization (on entry v, on exit y).
template <bool CHOL>
void dense_factor(int n, double* A, int32_t* info, int base, hipStream_t s, const int32_t* skip = nullptr,
                  double* y = nullptr) {
  // the first diagonal block on its own; every later one is factorized by
  // the trailing update of the previous block (fused, see k_blk_update)
  k_blk_diag<CHOL><<<1, 256, 0, s>>>(n, 0, A, info, base, skip, y);
  LAUNCHCHK();
  for (int b0 = 0; b0 < n; b0 += CB) {
    const int nb = std::min(CB, n - b0);
    const int rest = n - b0 - nb;
    if (rest > 0) {
      const int tasks = CHOL ? rest : 2 * rest;
      k_blk_panel<CHOL><<<cdiv(tasks, 4), 256, 0, s>>>(n, b0, A, info, skip);
      LAUNCHCHK();
      const int nt = cdiv(rest, CB);
      k_blk_update<CHOL><<<dim3(nt, nt), 256, 0, s>>>(n, b0, A, info, 1, base, skip, y);
      LAUNCHCHK();
    }
  }
}

void refactor(rpf_grid* h, hipStream_t s, const int32_t* skip = nullptr) {
  const Presolve& P = h->P;
  h->top_inv_ok = false;
  const size_t nnz = P.lu_col.size();
  k_gather_sum<<<cdiv(nnz, 256), 256, 0, s>>>((int)nnz, h->jx_sp, h->jx_s, h->rec, nullptr, h->luv, skip);
  LAUNCHCHK();
  const int maxrow = std::max(P.max_lu_row, 1);
  const int wv = h->rf_waves;
  const size_t shm = (size_t)wv * maxrow * sizeof(double);
  size_t pi = h->prof_on ? h->prof_begin(s) : 0;
  if (h->npacks > 0 && h->lds_rf > 0) {
    // the batched forward program's levels: rows outside the dense tails by
    // level, then the tails (finished right-looking)
    if (h->rf_recs_lds)
      k_rf_pack_lds<true><<<h->npacks, 1024, h->lds_rf, s>>>(h->pack_ptr, h->ptf_lev, h->ptf_lev_off, h->rf_rowrec,
                                                       h->lu_ptr, h->rf_ent, h->rf_entu0, h->upd_tgt, h->luv,
                                                       h->rdiag, 1e-14, h->piv_status, skip, h->ptl_off,
                                                       h->ptl_rows, h->rft_ptr, h->rf_tlrec);
    else
      k_rf_pack_lds<false><<<h->npacks, 1024, h->lds_rf, s>>>(h->pack_ptr, h->ptf_lev, h->ptf_lev_off, h->rf_rowrec,
                                                       h->lu_ptr, h->rf_ent, h->rf_entu0, h->upd_tgt, h->luv,
                                                       h->rdiag, 1e-14, h->piv_status, skip, h->ptl_off,
                                                       h->ptl_rows, h->rft_ptr, h->rf_tlrec);
    LAUNCHCHK();
  } else if (h->npacks > 0) {
    k_rf_pack<<<h->npacks, 64 * wv, shm, s>>>(h->pk_flev, h->pk_flev_off, h->pk_frows, h->lu_ptr, h->lu_col,
                                              h->lu_diag, h->upd_ptr, h->upd_tgt, h->luv, h->rdiag, maxrow,
                                              1e-14, h->piv_status, skip);
    LAUNCHCHK();
  }
  if (P.ntop > 0) {
    k_rf_top_ext<<<cdiv(P.ntop, wv), 64 * wv, shm, s>>>(P.t0, P.nx, h->lo_split, h->lu_ptr, h->lu_col, h->lu_diag,
                                                       h->upd_ptr, h->upd_tgt, h->luv, h->rdiag, maxrow,
                                                       h->piv_status, skip);
    LAUNCHCHK();
    const int64_t nd = (int64_t)P.ntop * P.ntop;
    k_fill_dbl<<<cdiv(nd, 256), 256, 0, s>>>(nd, h->dense_top, 0.0, skip);
    LAUNCHCHK();
    const int ne = (int)P.top_pos.size();
    k_dense_xfer<<<cdiv(ne, 256), 256, 0, s>>>(ne, h->top_pos, h->top_dense, h->luv, h->dense_top, 1, skip);
    LAUNCHCHK();
    // the dense top LU keeps its own word: a tiny pivot in the packs must not
    // stop it (its kernels return early once their info word is set)
    dense_factor<false>(P.ntop, h->dense_top, h->piv_status + 1, P.t0, s, skip);
    k_transpose<<<dim3(cdiv(P.ntop, 32), cdiv(P.ntop, 32)), dim3(32, 8), 0, s>>>(P.ntop, h->dense_top,
                                                                                 h->dense_topT, skip);
    LAUNCHCHK();
    k_dense_xfer<<<cdiv(ne, 256), 256, 0, s>>>(ne, h->top_pos, h->top_dense, h->luv, h->dense_top, 0, skip);
    LAUNCHCHK();
    // inverse diagonal blocks: J_x uses L (unit) and U; J_x^T uses U^T and L^T (unit)
    const dim3 gi(cdiv(P.ntop, CB), 2);
    k_top_diag_inv<<<gi, 256, 0, s>>>(P.ntop, h->dense_top, h->top_dinv, 1, 0, h->top_dinvT, skip);
    LAUNCHCHK();
  }
  if (h->prof_on) h->prof_end(2, pi, s);
  k_gather_pos<<<cdiv(nnz, 256), 256, 0, s>>>((int)nnz, h->lut_src, h->luv, h->lutv, skip);
  LAUNCHCHK();
}

// One right-hand side: the pack solves with level records when they fit in
// LDS, else the staged solves without them.
void pack_solve1(rpf_grid* h, bool fwd, bool unit, const double* val, double* X, int ld, double scale, int cls,
                 hipStream_t s, const int32_t* skip) {
  const Presolve& P = h->P;
  if (h->npacks == 0) return;
  const int ncols = 1;
  const size_t shm = h->lds_pack_s;
  const dim3 grd(h->npacks, 1);
  size_t pi = h->prof_on ? h->prof_begin(s) : 0;
  auto launch = [&](auto kern, const int32_t* lev, const int32_t* lev_off, const int32_t* rows, const int32_t* rp,
                    const int32_t* pos, const int16_t* ecol) {
    kern<<<grd, 256, shm, s>>>(h->pack_ptr, lev, lev_off, rows, rp, pos, ecol, h->lu_diag, h->up_split, h->lu_ptr,
                               h->lu_col, val, X, ld, ncols, scale, skip);
  };
  auto launch1 = [&](auto kern, const int32_t* lev, const int32_t* lev_off, const int8_t* lgs, const int32_t* rows,
                     const int32_t* rp, const int32_t* pos, const int16_t* ecol) {
    kern<<<h->npacks, 256, h->lds_pack1, s>>>(h->pack_ptr, lev, lev_off, lgs, rows, rp, pos, ecol, h->lu_diag,
                                               h->up_split, h->lu_ptr, h->lu_col, val, X, ld, scale, skip);
  };
  if (h->lds_pack1 <= h->lds_limit) {
    if (fwd) {
      if (unit)
        launch1(k_pack_solve_1<true, true>, h->pk_flev, h->pk_flev_off, h->pk_flg, h->pk_frows, h->pkf_rp,
                h->pkf_pos, h->pkf_col);
      else
        launch1(k_pack_solve_1<true, false>, h->pk_flev, h->pk_flev_off, h->pk_flg, h->pk_frows, h->pkf_rp,
                h->pkf_pos, h->pkf_col);
    } else {
      if (unit)
        launch1(k_pack_solve_1<false, true>, h->pk_blev, h->pk_blev_off, h->pk_blg, h->pk_brows, h->pkb_rp,
                h->pkb_pos, h->pkb_col);
      else
        launch1(k_pack_solve_1<false, false>, h->pk_blev, h->pk_blev_off, h->pk_blg, h->pk_brows, h->pkb_rp,
                h->pkb_pos, h->pkb_col);
    }
  } else if (fwd) {
    if (unit)
      launch(k_pack_solve_s<1, true, true>, h->pk_flev, h->pk_flev_off, h->pk_frows, h->pkf_rp, h->pkf_pos, h->pkf_col);
    else
      launch(k_pack_solve_s<1, true, false>, h->pk_flev, h->pk_flev_off, h->pk_frows, h->pkf_rp, h->pkf_pos, h->pkf_col);
  } else {
    if (unit)
      launch(k_pack_solve_s<1, false, true>, h->pk_blev, h->pk_blev_off, h->pk_brows, h->pkb_rp, h->pkb_pos, h->pkb_col);
    else
      launch(k_pack_solve_s<1, false, false>, h->pk_blev, h->pk_blev_off, h->pk_brows, h->pkb_rp, h->pkb_pos, h->pkb_col);
  }
  LAUNCHCHK();
  if (h->prof_on) h->prof_end(cls, pi, s);
  (void)P;
}

// Many right-hand sides: one workgroup of 1024 threads per (pack, 64 columns),
// solved in place in X.
template <int TW, bool SV>
void pack_solve_t(rpf_grid* h, bool fwd, bool unit, bool transposed, const double* val, double* X, int ld,
                  int ncols, double scale, hipStream_t s, const int32_t* skip, const PackFuse* fzp = nullptr) {
  const PackFuse fz = fzp ? *fzp : PackFuse{};
  const int ntiles = cdiv(ncols, TW);
  const dim3 grd(8 * cdiv(h->npacks, 8) * ntiles);   // see the XCD mapping in k_pack_solve_t
  const double* pv = fwd ? (transposed ? h->pkfvT : h->pkfv) : (transposed ? h->pkbvT : h->pkbv);
  // dense tail inverse of this solve: forward L_TT^-1 (J_x) or (U_TT^-1)^T
  // (J_x^T), backward U_TT^-1 (J_x) or (L_TT^-1)^T (J_x^T)
  const size_t n4 = (size_t)h->npacks * TAIL_MAX * TAIL_MAX;
  const int which = fwd ? (transposed ? 3 : 0) : (transposed ? 2 : 1);
  const double* tinv = h->tailM + which * n4;
  auto launch = [&](auto kern, const int32_t* lev, const int32_t* lev_off, const int32_t* rows, const int32_t* rp,
                    const int16_t* ecol) {
    kern<<<grd, h->packt_threads, h->lds_packt, s>>>(h->pack_ptr, lev, lev_off, rows, rp, ecol, pv, h->rdiag, h->up_split,
                                         h->lu_ptr, h->lu_col, val, X, ld, ncols, scale, h->npacks, ntiles,
                                         h->ptl_off, h->ptl_rows, tinv, skip, fz);
  };
  if (fwd) {
    if (unit) launch(k_pack_solve_t<TW, true, true, SV>, h->ptf_lev, h->ptf_lev_off, h->ptf_rows, h->ptf_rp, h->ptf_col);
    else launch(k_pack_solve_t<TW, true, false, SV>, h->ptf_lev, h->ptf_lev_off, h->ptf_rows, h->ptf_rp, h->ptf_col);
  } else {
    if (unit) launch(k_pack_solve_t<TW, false, true, SV>, h->ptb_lev, h->ptb_lev_off, h->ptb_rows, h->ptb_rp, h->ptb_col);
    else launch(k_pack_solve_t<TW, false, false, SV>, h->ptb_lev, h->ptb_lev_off, h->ptb_rows, h->ptb_rp, h->ptb_col);
  }
  LAUNCHCHK();
}

void pack_solve_g(rpf_grid* h, bool fwd, bool unit, bool transposed, const double* val, double* X, int ld,
                  int ncols, double scale, int cls, hipStream_t s, const int32_t* skip,
                  const PackFuse* fz = nullptr) {
  if (h->npacks == 0) return;
  if (h->tw_packt > 0) {
    size_t pi = h->prof_on ? h->prof_begin(s) : 0;
    if (h->tw_packt == 16) pack_solve_t<16, false>(h, fwd, unit, transposed, val, X, ld, ncols, scale, s, skip, fz);
    else if (h->sv_packt) pack_solve_t<8, true>(h, fwd, unit, transposed, val, X, ld, ncols, scale, s, skip, fz);
    else pack_solve_t<8, false>(h, fwd, unit, transposed, val, X, ld, ncols, scale, s, skip, fz);
    if (h->prof_on) h->prof_end(cls, pi, s);
    return;
  }
  dim3 grd(h->npacks, cdiv(ncols, 64));
  size_t pi = h->prof_on ? h->prof_begin(s) : 0;
  auto launch = [&](auto kern, const int32_t* lev, const int32_t* lev_off, const int32_t* rows) {
    kern<<<grd, 1024, h->lds_packg, s>>>(h->pack_ptr, lev, lev_off, rows, h->lu_ptr, h->lu_diag, h->lu_col, val, X,
                                         ld, ncols, scale, skip);
  };
  if (fwd) {
    if (unit) launch(k_pack_solve_g<true, true>, h->pk_flev, h->pk_flev_off, h->pk_frows);
    else launch(k_pack_solve_g<true, false>, h->pk_flev, h->pk_flev_off, h->pk_frows);
  } else {
    if (unit) launch(k_pack_solve_g<false, true>, h->pk_blev, h->pk_blev_off, h->pk_brows);
    else launch(k_pack_solve_g<false, false>, h->pk_blev, h->pk_blev_off, h->pk_brows);
  }
  LAUNCHCHK();
  if (h->prof_on) h->prof_end(cls, pi, s);
}

void pack_solve_any(rpf_grid* h, bool fwd, bool unit, bool transposed, const double* val, double* X,
                    int ld, int ncols, double scale, int cls, hipStream_t s, const int32_t* skip, const PackFuse* fz = nullptr) {
  if (ncols > 1) return pack_solve_g(h, fwd, unit, transposed, val, X, ld, ncols, scale, cls, s, skip, fz);
  pack_solve1(h, fwd, unit, val, X, ld, scale, cls, s, skip);
}

// Solves with both factors of J_x (transposed = false): X <- U^{-1} L^{-1}
// (scale X), or of J_x^T (transposed = true): X <- L^{-T} U^{-T} (scale X).
// Four launches: packs forward, right-hand side of the top rows (pack
// contributions), dense top part forward + backward, packs backward.
// rf (forward, J_x only): the first pack solve forms R = -J_u V itself
// (the caller has formed the top rows of R).  With the LDS-tile pack solves
// the backward pack solve subtracts the pack rows' top-column products
// itself.
void solve_pair(rpf_grid* h, bool transposed, double* X, int ld, int ncols, double scale, hipStream_t s,
                const int32_t* skip = nullptr, const PackFuse* rf = nullptr) {
  const Presolve& P = h->P;
  const double* val = transposed ? h->lutv : h->luv;
  // forward factor: L (unit) or U^T (non-unit); backward: U (non-unit) or L^T (unit)
  const bool fwd_unit = !transposed;
  const int cls = ncols > 1 ? 0 : 1;
  const int twt = ncols == 1 ? 1 : h->tw_top;
  pack_solve_any(h, true, fwd_unit, transposed, val, X, ld, ncols, scale, cls, s, skip, rf);
  const bool fuse_top = ncols > 1 && h->tw_packt > 0 && h->npacks > 0;
  if (P.ntop > 0) {
    size_t pi = h->prof_on ? h->prof_begin(s) : 0;
    // single right-hand sides of the power flow and adjoint: lanes split a
    // row's entries; the Hessian products (any width) sum each column in the
    // same fixed order
    const bool single = ncols == 1 && !h->top_inv_ok && (size_t)P.ntop * sizeof(double) <= 64 * 1024;
    if (single) {
      k_top_rhs1<<<cdiv(P.ntop, 4), 256, 0, s>>>(P.t0, P.nx, h->lo_split, h->lu_ptr, h->lu_col, val, X, ld, scale,
                                                 skip);
    } else if (ncols > 64) {
      k_top_rhs_w<2><<<dim3(cdiv(ncols, 128), cdiv(P.ntop, 4)), 256, 0, s>>>(P.t0, P.nx, h->lo_split, h->lu_ptr,
                                                                            h->lu_col, val, X, ld, ncols, scale,
                                                                            skip);
    } else if (ncols > 1) {
      k_top_rhs_w<1><<<dim3(cdiv(ncols, 64), cdiv(P.ntop, 4)), 256, 0, s>>>(P.t0, P.nx, h->lo_split, h->lu_ptr,
                                                                           h->lu_col, val, X, ld, ncols, scale,
                                                                           skip);
    } else {
      const dim3 rb(1, 256);
      k_top_rhs<<<dim3(1, cdiv(P.ntop, 256)), rb, 0, s>>>(P.t0, P.nx, h->lo_split, h->lu_ptr, h->lu_col, val, X,
                                                           ld, ncols, scale, skip);
    }
    LAUNCHCHK();
    if (h->top_inv_ok) {
      // one dense product with the inverse (k-major: S^-T gives S^-1 X)
      const double* A = transposed ? h->top_inv : h->top_invT;
      const int nt = std::min(1024, 64 * cdiv(P.ntop, 64));
      if (ncols >= 2048)
        // wide batches: four columns per workgroup, half the L2 reads of the
        // inverse (measured at 2889 columns: 4 faster than 2 or 8)
        k_top_inv_apply<4><<<cdiv(ncols, 4), nt, (size_t)P.ntop * 4 * sizeof(double), s>>>(P.t0, P.ntop, A, X, ld,
                                                                                           ncols, skip);
      else if (ncols > 1)
        // two columns per workgroup: more workgroups to hide the L2 latency
        // of the inverse's rows (measured up to 1024 columns: 2 faster than
        // 4 or 8)
        k_top_inv_apply<2><<<cdiv(ncols, 2), nt, (size_t)P.ntop * 2 * sizeof(double), s>>>(P.t0, P.ntop, A, X, ld,
                                                                                           ncols, skip);
      else
        k_top_inv_apply<1><<<ncols, nt, (size_t)P.ntop * sizeof(double), s>>>(P.t0, P.ntop, A, X, ld, ncols, skip);
      LAUNCHCHK();
    } else {
      const double* M = transposed ? h->dense_topT : h->dense_top;
      const double* dinv = transposed ? h->top_dinvT : h->top_dinv;
      if (single) {
        k_top_solve1<<<1, 1024, (size_t)P.ntop * sizeof(double), s>>>(P.t0, P.nx, M, dinv, X, ld, skip);
      } else {
        const size_t shm = (size_t)P.ntop * twt * sizeof(double);
        k_top_dense<<<cdiv(ncols, twt), 256, shm, s>>>(P.t0, P.nx, M, dinv, X, ld, ncols, twt, skip);
      }
      LAUNCHCHK();
    }
    if (ncols > 1 && h->tw_packt > 0 && h->npacks > 0 && !fuse_top) {
      // the LDS-tile pack solves expect the top products already subtracted
      if (h->n_topmul_rows > 0) {
        const int nr = h->n_topmul_rows;
        if (ncols > 64)
          k_pack_topmul_w<2><<<dim3(cdiv(ncols, 128), cdiv(nr, 4)), 256, 0, s>>>(nr, h->topmul_rows, h->up_split,
                                                                                h->lu_ptr, h->lu_col, val, X, ld,
                                                                                ncols, skip);
        else
          k_pack_topmul_w<1><<<dim3(cdiv(ncols, 64), cdiv(nr, 4)), 256, 0, s>>>(nr, h->topmul_rows, h->up_split,
                                                                               h->lu_ptr, h->lu_col, val, X, ld,
                                                                               ncols, skip);
        LAUNCHCHK();
      }
    }
    if (h->prof_on) h->prof_end(cls == 0 ? 5 : cls, pi, s);
  }
  PackFuse bf;
  if (fuse_top && P.ntop > 0) {
    bf.tmoff = h->tm_off;
    bf.tmrows = h->topmul_rows;
  }
  pack_solve_any(h, false, !fwd_unit, transposed, val, X, ld, ncols, 1.0, cls, s, skip,
                 fuse_top ? &bf : nullptr);
}

// Y = alpha A1 X1 (+ Yadd); with A2, then Y = A2 X2 + that (one pass).
void spmm_terms(rpf_grid* h, int nrows, const SpTerm& A1, const SpTerm* A2, int ncols, double alpha,
                const double* Yadd, int ldya, double* Y, int ldy, hipStream_t s) {
  size_t pi = h->prof_on ? h->prof_begin(s) : 0;
  const SpTerm B2 = A2 ? *A2 : A1;
  // two columns per lane once a row has more than one wavefront's worth
  const dim3 g2(cdiv(ncols, 128), cdiv(nrows, 4)), g1(cdiv(ncols, 64), cdiv(nrows, 4));
  if (ncols > 64 && A2)
    k_spmm<2, true><<<g2, 256, 0, s>>>(nrows, A1, B2, ncols, alpha, 1.0, Yadd, ldya, Y, ldy,
                                                 h->skipw);
  else if (ncols > 64)
    k_spmm<2, false><<<g2, 256, 0, s>>>(nrows, A1, B2, ncols, alpha, 1.0, Yadd, ldya, Y, ldy,
                                                 h->skipw);
  else if (A2)
    k_spmm<1, true><<<g1, 256, 0, s>>>(nrows, A1, B2, ncols, alpha, 1.0, Yadd, ldya, Y, ldy,
                                                 h->skipw);
  else
    k_spmm<1, false><<<g1, 256, 0, s>>>(nrows, A1, B2, ncols, alpha, 1.0, Yadd, ldya, Y, ldy,
                                                 h->skipw);
  LAUNCHCHK();
  if (h->prof_on) h->prof_end(3, pi, s);
}

void spmm(rpf_grid* h, int nrows, const int32_t* ptr, const int32_t* col, const double* val,
          const int32_t* valpos, const double* xscale, const double* X, int ldx, int ncols, double alpha,
          const double* Yadd, int ldya, double* Y, int ldy, hipStream_t s) {
  const SpTerm A{ptr, col, val, valpos, xscale, X, ldx};
  spmm_terms(h, nrows, A, nullptr, ncols, alpha, Yadd, ldya, Y, ldy, s);
}

// step = -(L L^T)^{-1} rhs with the dense Cholesky factor L (row-major n x n,
// lower triangle): one workgroup per two blocks of CB rows in each
// direction.
// Scratch: flags [2 cdiv(n, CB)] (cleared here by a kernel), dinv
// [cdiv(n, CB) 2 CB CB], work [n].
void chol_solve_ws(int n, const double* L, const double* rhs, double* step, int32_t* info, int32_t* flags,
                   double* dinv, double* work, hipStream_t s) {
  const int nblk = cdiv(n, CB);
  k_fill_int<<<cdiv(2 * nblk, 256), 256, 0, s>>>(2 * nblk, flags, 0);
  LAUNCHCHK();
  // inverses of the diagonal blocks (skipped when the factorization failed)
  k_top_diag_inv<<<dim3(nblk, 1), 256, 0, s>>>(n, L, dinv, 0, 0, nullptr, info);
  LAUNCHCHK();
  const int nwg = cdiv(n, 2 * CB);   // two blocks per workgroup
  k_chol_fwd<<<nwg, 512, 0, s>>>(n, L, dinv, rhs, work, flags, info);
  LAUNCHCHK();
  k_chol_bwd<<<nwg, 512, 0, s>>>(n, L, dinv, work, step, flags + nblk, info);
  LAUNCHCHK();
}

void chol_solve(rpf_grid* h, int n, const double* L, const double* rhs, double* step, int32_t* info,
                hipStream_t s) {
  chol_solve_ws(n, L, rhs, step, info, h->chol_flags, h->chol_dinv, h->chol_work, s);
}

// K = L L^T in place and step = -K^{-1} rhs with the forward solve fused
// into the factorization (y = -L^{-1} rhs in work), then L^T step = y.
// Scratch as chol_solve_ws.
void factor_then_solve(int n, double* K, const double* rhs, double* step, int32_t* info, int32_t* flags,
                       double* dinv, double* work, hipStream_t s) {
  const int nblk = cdiv(n, CB);
  k_neg_copy<<<cdiv(n, 256), 256, 0, s>>>(n, rhs, work);
  LAUNCHCHK();
  dense_factor<true>(n, K, info, 0, s, nullptr, work);
  k_fill_int<<<cdiv(nblk, 256), 256, 0, s>>>(nblk, flags + nblk, 0);
  LAUNCHCHK();
  // inverses of the diagonal blocks (skipped when the factorization failed)
  k_top_diag_inv<<<dim3(nblk, 1), 256, 0, s>>>(n, K, dinv, 0, 0, nullptr, info);
  LAUNCHCHK();
  k_chol_bwd<<<cdiv(n, 2 * CB), 512, 0, s>>>(n, K, dinv, work, step, flags + nblk, info);
  LAUNCHCHK();
}

// The dense step K = (K + K^T)/2 + diag + delta I = L L^T, step = -K^{-1} rhs,
// on `s` with the given triangular-solve scratch.
void factor_solve_ws(int n, double* K, const double* diag, double delta, const double* rhs, double* step,
                     int32_t* info, int32_t* flags, double* dinv, double* work, hipStream_t s) {
  k_fill_int<<<1, 1, 0, s>>>(1, info, 0);
  LAUNCHCHK();
  k_symmetrize<<<dim3(cdiv(n, 32), cdiv(n, 32)), dim3(32, 8), 0, s>>>(n, K, diag, delta);
  LAUNCHCHK();
  factor_then_solve(n, K, rhs, step, info, flags, dinv, work, s);
}

ALArgs al_args(rpf_grid* h, const double* u, const double* pd, const double* qd, const double* s,
               const double* y, double rho, const double* sigma) {
  const Presolve& P = h->P;
  ALArgs A;
  A.nb = P.nb; A.nl = P.nl; A.npq = P.npq; A.npv = P.npv; A.ng = P.ng; A.m = P.m; A.nx = P.nx; A.nu = P.nu;
  A.ref = P.ref; A.gen_ref = P.gen_at[P.ref];
  A.base = P.base_mva; A.rho = rho; A.sigf = sigma;
  A.pq = h->pq; A.pv = h->pv; A.gen_pidx = h->gen_pidx; A.pv_gen = h->pv_gen;
  A.c2 = h->c2; A.c1 = h->c1; A.c0 = h->c0;
  A.rec = h->rec; A.Pbus = h->Pbus; A.Qbus = h->Qbus; A.vm = h->vm;
  A.pd = pd; A.qd = qd; A.u = u; A.s = s; A.y = y; A.sigma_c = sigma + 1;
  return A;
}

VarArgs var_args(rpf_grid* h, const double* u, const double* sigma) {
  const Presolve& P = h->P;
  VarArgs V;
  V.nvar = P.nvar; V.nx = P.nx; V.npq = P.npq; V.npv = P.npv; V.nl = P.nl;
  V.base = P.base_mva; V.sigf = sigma;
  V.kind = h->var_kind; V.aux = h->var_aux; V.pv_gen = h->pv_gen; V.pv = h->pv; V.rowP = h->rowP;
  V.c2 = h->c2; V.c1 = h->c1; V.u = u;
  return V;
}

void bus_injections(rpf_grid* h, hipStream_t s) {
  const Presolve& P = h->P;
  k_gather_sum<<<cdiv(P.nb, 256), 256, 0, s>>>(P.nb, h->pb_ptr, h->pb_src, h->rec, nullptr, h->Pbus, nullptr);
  LAUNCHCHK();
  k_gather_sum<<<cdiv(P.nb, 256), 256, 0, s>>>(P.nb, h->pb_ptr, h->qb_src, h->rec, nullptr, h->Qbus, nullptr);
  LAUNCHCHK();
}

// One batch of reduced Hessian-vector products at the cached point.
// V (ldv) or, when V is null, identity columns j0.. of the n_u identity.
// Proposition 2 on one batch of directions, in workspace slot ws (D, Y, T).
// With J (ldj), also the batch's columns j0 .. j0 + B of the reduced
// Jacobian of the constraints from the same Z (no extra solves); with HV
// null, only that (the adjoint half is skipped).
void hvp_batch(rpf_grid* h, const double* V, int ldv, int j0, int B, double* HV, int ldhv, hipStream_t s,
               int ws = 0, double* J = nullptr, int ldj = 0) {
  const Presolve& P = h->P;
  const int ld = B;
  double* const D = h->Dk[ws];
  double* const Y = h->Yk[ws];
  double* const T = h->Tk[ws];
  double* Dx = D;
  double* Du = D + (size_t)P.nx * ld;
  dim3 blk(64, 4);
  if (V) {
    k_copy_block<<<dim3(cdiv(B, 64), cdiv(P.nu, 4)), blk, 0, s>>>(P.nu, B, V, ldv, Du, ld, h->skipw);
  } else {
    k_identity_block<<<dim3(cdiv(B, 64), cdiv(P.nu, 4)), blk, 0, s>>>(P.nu, B, j0, Du, ld, h->skipw);
  }
  LAUNCHCHK();
  // R = -J_u V, then Z = U^{-1} L^{-1} R.  With the LDS-tile pack solves
  // the first pack solve forms the pack rows of R itself; only the top rows
  // are formed here
  if (h->tw_packt > 0 && h->npacks > 0 && B > 1) {
    if (P.ntop > 0)
      spmm(h, P.ntop, h->ju_ptr + P.t0, h->ju_col, h->juv, nullptr, nullptr, Du, ld, B, -1.0, nullptr, 0,
           Dx + (size_t)P.t0 * ld, ld, s);
    PackFuse rf;
    rf.jp = h->ju_ptr;
    rf.jc = h->ju_col;
    rf.jv = h->juv;
    rf.V = Du;
    rf.ldv = ld;
    solve_pair(h, false, Dx, ld, B, 1.0, s, h->skipw, &rf);
  } else {
    spmm(h, P.nx, h->ju_ptr, h->ju_col, h->juv, nullptr, nullptr, Du, ld, B, -1.0, nullptr, 0, Dx, ld, s);
    solve_pair(h, false, Dx, ld, B, 1.0, s, h->skipw);
  }
  // Y = K [Z; V] + G^T diag(kappa) G [Z; V]
  // (T = G [Z; V] first; then both terms of Y in one pass over its rows)
  spmm(h, P.nr1, h->G_ptr, h->G_col, h->Gv, nullptr, nullptr, D, ld, B, 1.0, nullptr, 0, T, ld, s);
  if (J) {
    k_cjac_batch<<<dim3(cdiv(B, 64), cdiv(P.m, 4)), dim3(64, 4), 0, s>>>(P.nl, P.npq, P.m, B, h->br_f, h->br_t,
                                                                       h->th_var, h->v_var, h->pq, h->rec, D, ld,
                                                                       T, ld, J, ldj, j0);
    LAUNCHCHK();
  }
  if (!HV) return;
  {
    const SpTerm Kt{h->K_ptr, h->K_col, h->Kv, nullptr, nullptr, D, ld};
    const SpTerm Gk{h->Gt_ptr, h->Gt_col, h->Gv, h->Gt_pos, h->kappa, T, ld};
    spmm_terms(h, P.nvar, Kt, &Gk, B, 1.0, nullptr, 0, Y, ld, s);
  }
  // Psi = -J_x^{-T} Y_x  (U^T then L^T)
  solve_pair(h, true, Y, ld, B, -1.0, s, h->skipw);
  // HV = Y_u + J_u^T Psi
  spmm(h, P.nu, h->jut_ptr, h->jut_col, h->juv, h->jut_pos, nullptr, Y, ld, B, 1.0, Y + (size_t)P.nx * ld,
       ld, HV, ldhv, s);
}

// Newton power flow on h->xi with `iters` predicated steps and no host
// synchronisation: done[0] is raised to 1 when ||g||_2 < tol (to 2 when the
// residual is not finite) and every later kernel of the loop returns at
// once; count[0] counts the steps taken and resid[0] holds the last
// residual norm.  A nonzero done[0] on entry skips the whole solve.
void pf_device(rpf_grid* h, const double* u, const double* pd, const double* qd, int iters, double tol,
               int32_t* done, int32_t* count, double* resid, hipStream_t s) {
  const Presolve& P = h->P;
  const int nblk = cdiv(P.nx, 256);
  // pivot words start clear for every power flow (the dense top LU skips
  // its work while its word is set)
  k_fill_int<<<1, 4, 0, s>>>(4, h->piv_status, 0);
  LAUNCHCHK();
  for (int k = 0; k <= iters; ++k) {
    state_and_records(h, u, s, done);
    k_residual<<<nblk, 256, 0, s>>>(P.nx, h->g_sp, h->g_s, h->rec, h->row_bus, h->row_isq, h->row_pvar, pd, qd, u,
                                    h->g, h->partial, done);
    LAUNCHCHK();
    k_reduce_final<<<1, 1024, 0, s>>>(nblk, h->partial, resid, 1, tol, done, done);
    LAUNCHCHK();
    if (k == iters) break;
    refactor(h, s, done);
    k_copy_vec<<<nblk, 256, 0, s>>>(P.nx, h->g, h->d, done);
    LAUNCHCHK();
    solve_pair(h, false, h->d, 1, 1, 1.0, s, done);
    k_axpy<<<nblk, 256, 0, s>>>(P.nx, -1.0, h->d, h->xi, done);
    LAUNCHCHK();
    k_count<<<1, 1, 0, s>>>(done, count);
    LAUNCHCHK();
  }
}

template <class F>
int guard(F&& f) {
  try {
    return f();
  } catch (const HipError& e) {
    return set_err(RPF_EHIP, e.what());
  } catch (const std::bad_alloc&) {
    return set_err(RPF_ENOMEM, "device allocation failed");
  } catch (const std::exception& e) {
    return set_err(RPF_EINVAL, e.what());
  }
}

}  // namespace

namespace {
GridData grid_from_desc(const rpf_grid_desc* desc) {
  if (!desc) throw std::runtime_error("desc is NULL");
  if (!desc->bus_type || !desc->br_from || !desc->br_to || !desc->br_r || !desc->br_x || !desc->br_b ||
      !desc->gen_bus || !desc->c2 || !desc->c1 || !desc->c0)
    throw std::runtime_error("grid description has a NULL array");
  if (desc->nb < 2 || desc->nl < 1 || desc->ng < 1) throw std::runtime_error("grid needs nb >= 2, nl >= 1, ng >= 1");
  if (!(desc->base_mva > 0.0)) throw std::runtime_error("base_mva must be positive");
  GridData G;
  G.nb = desc->nb; G.nl = desc->nl; G.ng = desc->ng; G.base_mva = desc->base_mva;
  G.bus_type.assign(desc->bus_type, desc->bus_type + G.nb);
  G.br_from.assign(desc->br_from, desc->br_from + G.nl);
  G.br_to.assign(desc->br_to, desc->br_to + G.nl);
  G.br_r.assign(desc->br_r, desc->br_r + G.nl);
  G.br_x.assign(desc->br_x, desc->br_x + G.nl);
  G.br_b.assign(desc->br_b, desc->br_b + G.nl);
  G.gen_bus.assign(desc->gen_bus, desc->gen_bus + G.ng);
  G.c2.assign(desc->c2, desc->c2 + G.ng);
  G.c1.assign(desc->c1, desc->c1 + G.ng);
  G.c0.assign(desc->c0, desc->c0 + G.ng);
  return G;
}
}  // namespace

extern "C" {

const char* rpf_last_error(void) { return g_err.c_str(); }

int rpf_profile_enable(rpf_grid* h, int32_t enable) {
  if (!h) return set_err(RPF_EINVAL, "grid is NULL");
  h->prof_on = enable != 0;
  return RPF_OK;
}

int rpf_profile_read_busy(rpf_grid* h, double* ms, int64_t* launches, double* busy_ms, int32_t reset) {
  if (!h || !ms || !launches) return set_err(RPF_EINVAL, "NULL argument");
  return guard([&]() -> int {
    std::vector<std::vector<std::pair<double, double>>> iv(RPF_PROF_CLASSES);
    for (int c = 0; c < RPF_PROF_CLASSES; ++c) {
      ms[c] = 0.0;
      launches[c] = 0;
      if (busy_ms) busy_ms[c] = 0.0;
    }
    const hipEvent_t ref = h->ev_marks.empty() ? nullptr : h->ev_pool[h->ev_marks.front().second];
    for (auto& mk : h->ev_marks) {
      HIPCHK(hipEventSynchronize(h->ev_pool[mk.second + 1]));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, h->ev_pool[mk.second], h->ev_pool[mk.second + 1]));
      ms[mk.first] += t;
      launches[mk.first] += 1;
      if (busy_ms) {
        // interval of this launch relative to the first recorded event
        float a = 0.f, b = 0.f;
        HIPCHK(hipEventElapsedTime(&a, ref, h->ev_pool[mk.second]));
        HIPCHK(hipEventElapsedTime(&b, ref, h->ev_pool[mk.second + 1]));
        iv[mk.first].push_back({(double)a, (double)b});
      }
    }
    if (busy_ms) {
      for (int c = 0; c < RPF_PROF_CLASSES; ++c) {
        auto& v = iv[c];
        std::sort(v.begin(), v.end());
        double total = 0.0, lo = 0.0, hi = 0.0;
        bool open = false;
        for (auto& x : v) {
          if (!open || x.first > hi) {
            if (open) total += hi - lo;
            lo = x.first;
            hi = x.second;
            open = true;
          } else {
            hi = std::max(hi, x.second);
          }
        }
        if (open) total += hi - lo;
        busy_ms[c] = total;
      }
    }
    if (reset) {
      h->ev_marks.clear();
      h->ev_used = 0;
    }
    return RPF_OK;
  });
}

int rpf_profile_read(rpf_grid* h, double* ms, int64_t* launches, int32_t reset) {
  return rpf_profile_read_busy(h, ms, launches, nullptr, reset);
}


// packs of independent subtrees: at most RPF_SUBTREE_MAX rows (default 1024,
// sized for 160 KB of LDS per workgroup)
static int subtree_max() {
  int smax = 1024;
  if (const char* e = std::getenv("RPF_SUBTREE_MAX")) smax = std::max(1, std::min(32767, std::atoi(e)));
  return smax;
}

// rows of the dense tail of each pack in the batched solves (0 = none)
static int tail_max() {
  int t = 128;
  if (const char* e = std::getenv("RPF_TAIL_MAX")) t = std::max(0, std::min(128, std::atoi(e)));
  return t;
}

int rpf_presolve_info(const rpf_grid_desc* desc, int64_t* o) {
  if (!o) return set_err(RPF_EINVAL, "out is NULL");
  return guard([&]() -> int {
    Presolve P = build_presolve(grid_from_desc(desc), subtree_max(), tail_max());
    PresolveStats st = stats(P);
    int64_t v[20] = {P.nx, P.nu, P.m, st.nnz_jx, st.nnz_lu, st.nlev_lo, st.nlev_up, st.max_lu_row,
                     st.refactor_updates, st.nnz_ju, st.nnz_k, st.nnz_g, st.npacks, st.ntop,
                     st.max_pack_levels, st.top_levels, st.max_tail_fwd_levels, st.max_tail_bwd_levels,
                     st.tail_rows, P.tail_max};
    std::memcpy(o, v, sizeof(v));
    return RPF_OK;
  });
}

int rpf_presolve_pattern(const rpf_grid_desc* desc, int32_t* perm, int32_t* lu_ptr, int32_t* lu_col) {
  return guard([&]() -> int {
    Presolve P = build_presolve(grid_from_desc(desc), subtree_max(), tail_max());
    if (perm) std::copy(P.x_int2paper.begin(), P.x_int2paper.end(), perm);
    if (lu_ptr) std::copy(P.lu_ptr.begin(), P.lu_ptr.end(), lu_ptr);
    if (lu_col) std::copy(P.lu_col.begin(), P.lu_col.end(), lu_col);
    return RPF_OK;
  });
}

int rpf_grid_create(const rpf_grid_desc* desc, int32_t max_batch, rpf_grid** out) {
  if (!out) return set_err(RPF_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_batch < 1) return set_err(RPF_EINVAL, "max_batch must be >= 1");
  return guard([&]() -> int {
    GridData G0 = grid_from_desc(desc);
    rpf_grid* h = new rpf_grid();
    try {
      h->G = std::move(G0);
      const GridData& G = h->G;
      h->P = build_presolve(G, subtree_max(), tail_max());
      h->max_batch = max_batch;
      if ((int64_t)h->P.nvar * max_batch >= (int64_t)1 << 31)
        throw std::runtime_error("n_var * max_batch must stay below 2^31");
      setup(h);
      const char* tr = std::getenv("RPF_TRACE");
      h->trace_on = tr && *tr && std::strcmp(tr, "0") != 0;
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return RPF_OK;
  });
}

void rpf_grid_destroy(rpf_grid* grid) { delete grid; }

int rpf_dims(const rpf_grid* h, int32_t* nx, int32_t* nu, int32_t* m) {
  if (!h) return set_err(RPF_EINVAL, "grid is NULL");
  if (nx) *nx = h->P.nx;
  if (nu) *nu = h->P.nu;
  if (m) *m = h->P.m;
  return RPF_OK;
}

int rpf_structure(const rpf_grid* h, int64_t* o) {
  if (!h || !o) return set_err(RPF_EINVAL, "NULL argument");
  PresolveStats st = stats(h->P);
  o[0] = st.nnz_jx; o[1] = st.nnz_lu; o[2] = st.nlev_lo; o[3] = st.nlev_up; o[4] = st.max_lu_row;
  o[5] = st.refactor_updates; o[6] = st.nnz_ju; o[7] = st.nnz_k; o[8] = st.nnz_g; o[9] = h->max_batch;
  return RPF_OK;
}

int rpf_pf_solve(rpf_grid* h, const double* u, const double* pd, const double* qd, double* x, double tol,
                 int32_t max_iter, int32_t* status, double* resid, rpf_stream_t stream) {
  if (!h || !u || !pd || !qd || !x || !status || !resid) return set_err(RPF_EINVAL, "NULL argument");
  if (max_iter < 0 || max_iter > 100) return set_err(RPF_EINVAL, "max_iter must be in [0, 100]");
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    Traced trace_scope(h, "rpf_pf_solve", s, (long long)max_iter);
    const Presolve& P = h->P;
    h->have_point = false;
    x_in(h, x, s);
    // flag[0]: predication word of the Newton loop, flag[1]: steps taken
    k_fill_int<<<1, 4, 0, s>>>(4, h->flag, 0);
    LAUNCHCHK();
    pf_device(h, u, pd, qd, max_iter, tol, h->flag, h->flag + 1, h->resid_d, s);
    k_pf_status<<<1, 1, 0, s>>>(status, h->flag + 1, h->flag, h->piv_status, h->x_i2p, h->resid_d, resid);
    LAUNCHCHK();
    k_permute_scatter<<<cdiv(P.nx, 256), 256, 0, s>>>(P.nx, h->x_i2p, h->xi, x, nullptr);
    LAUNCHCHK();
    return RPF_OK;
  });
}

int rpf_al_objective(rpf_grid* h, const double* x, const double* u, const double* pd, const double* qd,
                     const double* sv, const double* y, double rho, const double* sigma, double* phi,
                     double* c, rpf_stream_t stream) {
  if (!h || !x || !u || !pd || !qd || !sv || !y || !sigma || !phi) return set_err(RPF_EINVAL, "NULL argument");
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    Traced trace_scope(h, "rpf_al_objective", s);
    const Presolve& P = h->P;
    x_in(h, x, s);
    state_and_records(h, u, s);
    bus_injections(h, s);
    ALArgs A = al_args(h, u, pd, qd, sv, y, rho, sigma);
    k_constraints<<<cdiv(P.m + P.ng, 256), 256, 0, s>>>(A, c ? c : h->cvec, h->wvec, h->terms);
    LAUNCHCHK();
    k_reduce_final<<<1, 1024, 0, s>>>(P.m + P.ng, h->terms, phi, 0, 0.0, nullptr, nullptr);
    LAUNCHCHK();
    return RPF_OK;
  });
}

}  // extern "C"

namespace {

// Reduced gradient at the state already in h->xi (internal order); caches
// the point for the Hessian products.  grad and lambda (paper order) may be
// null.
void gradient_core(rpf_grid* h, const double* u, const double* pd, const double* qd, const double* sv,
                   const double* y, double rho, const double* sigma, double* grad, double* lambda, hipStream_t s) {
  const Presolve& P = h->P;
  h->have_point = false;
  state_and_records(h, u, s);
  bus_injections(h, s);
  ALArgs A = al_args(h, u, pd, qd, sv, y, rho, sigma);
  VarArgs V = var_args(h, u, sigma);
  k_constraints<<<cdiv(P.m + P.ng, 256), 256, 0, s>>>(A, h->cvec, h->wvec, nullptr);
  LAUNCHCHK();
  const int nbw = cdiv(P.nb + 2 + P.npv, 256);
  // d phi / d(variables) through branch-local gradients
  k_bus_weights<<<nbw, 256, 0, s>>>(A, h->wvec, nullptr, h->rowP, h->rowQ, h->bus_pvpos, h->a, h->b, h->kappa);
  LAUNCHCHK();
  k_branch_second<<<cdiv(P.nl, 256), 256, 0, s>>>(P.nl, h->br_f, h->br_t, h->br_r, h->br_x, h->br_b, h->th,
                                                   h->vm, h->rec, h->a, h->b, h->wvec, sigma + 1, rho, h->wrec);
  LAUNCHCHK();
  k_var_grad<<<cdiv(P.nvar, 256), 256, 0, s>>>(V, h->vg_sp, h->vg_s, h->wrec, h->wvec, nullptr, h->varg);
  LAUNCHCHK();
  // J_x factorized at x; lambda: U^T w = -d_x phi, L^T lambda = w
  k_fill_int<<<1, 4, 0, s>>>(4, h->piv_status, 0);
  LAUNCHCHK();
  refactor(h, s);
  // factor values in the batched programs' order, and the inverses of the
  // packs' dense tails
  if (h->tw_packt > 0) {
    const int nf = (int)P.ptf_pos.size(), nb_ = (int)P.ptb_pos.size();
    if (nf > 0) {
      k_gather_pos<<<cdiv(nf, 256), 256, 0, s>>>(nf, h->ptf_pos, h->luv, h->pkfv, nullptr);
      LAUNCHCHK();
      k_gather_pos<<<cdiv(nf, 256), 256, 0, s>>>(nf, h->ptf_pos, h->lutv, h->pkfvT, nullptr);
      LAUNCHCHK();
    }
    if (nb_ > 0) {
      k_gather_pos<<<cdiv(nb_, 256), 256, 0, s>>>(nb_, h->ptb_pos, h->luv, h->pkbv, nullptr);
      LAUNCHCHK();
      k_gather_pos<<<cdiv(nb_, 256), 256, 0, s>>>(nb_, h->ptb_pos, h->lutv, h->pkbvT, nullptr);
      LAUNCHCHK();
    }
    const int nte = (int)P.ptl_pos.size();
    if (nte > 0 && h->npacks > 0) {
      const int64_t na = (int64_t)h->npacks * 2 * TAIL_MAX * TAIL_MAX;
      k_fill_dbl<<<cdiv(na, 256), 256, 0, s>>>(na, h->tailA, 0.0, nullptr);
      LAUNCHCHK();
      k_tail_gather<<<cdiv(nte, 256), 256, 0, s>>>(nte, h->ptl_eoff, h->npacks, h->ptl_pos, h->ptl_dense, h->ptl_off,
                                                   h->luv, h->tailA, nullptr);
      LAUNCHCHK();
      k_tail_diag_inv<<<dim3(h->npacks, 2, TAIL_MAX / CB), 256, 0, s>>>(h->ptl_off, h->tailA, h->tailM, h->npacks,
                                                                       nullptr);
      LAUNCHCHK();
      k_tail_offdiag<<<dim3(h->npacks, 2), 256, 0, s>>>(h->ptl_off, h->tailA, h->tailM, h->npacks, nullptr);
      LAUNCHCHK();
    }
  }
  k_copy_vec<<<cdiv(P.nx, 256), 256, 0, s>>>(P.nx, h->varg, h->lam, nullptr);
  LAUNCHCHK();
  solve_pair(h, true, h->lam, 1, 1, -1.0, s);
  // gradient of l = phi + lambda^T g: its control part is the reduced gradient
  k_bus_weights<<<nbw, 256, 0, s>>>(A, h->wvec, h->lam, h->rowP, h->rowQ, h->bus_pvpos, h->a, h->b, h->kappa);
  LAUNCHCHK();
  k_branch_second<<<cdiv(P.nl, 256), 256, 0, s>>>(P.nl, h->br_f, h->br_t, h->br_r, h->br_x, h->br_b, h->th,
                                                   h->vm, h->rec, h->a, h->b, h->wvec, sigma + 1, rho, h->wrec);
  LAUNCHCHK();
  k_var_grad<<<cdiv(P.nvar, 256), 256, 0, s>>>(V, h->vg_sp, h->vg_s, h->wrec, h->wvec, h->lam, h->varg);
  LAUNCHCHK();
  if (grad) {
    k_copy_vec<<<cdiv(P.nu, 256), 256, 0, s>>>(P.nu, h->varg + P.nx, grad, nullptr);
    LAUNCHCHK();
  }
  if (lambda) {
    k_permute_scatter<<<cdiv(P.nx, 256), 256, 0, s>>>(P.nx, h->x_i2p, h->lam, lambda, nullptr);
    LAUNCHCHK();
  }
  // cached point for the Hessian products
  k_gather_sum<<<cdiv(P.K_col.size(), 256), 256, 0, s>>>((int)P.K_col.size(), h->K_sp, h->K_s, h->wrec, nullptr,
                                                          h->Kv, nullptr);
  LAUNCHCHK();
  k_k_diag<<<cdiv(P.nvar, 256), 256, 0, s>>>(V, h->K_diag, sigma + 1, rho, h->Kv);
  LAUNCHCHK();
  k_gather_sum<<<cdiv(P.ju_col.size(), 256), 256, 0, s>>>((int)P.ju_col.size(), h->ju_sp, h->ju_s, h->rec,
                                                           h->ju_const, h->juv, nullptr);
  LAUNCHCHK();
  k_gather_sum<<<cdiv(P.G_col.size(), 256), 256, 0, s>>>((int)P.G_col.size(), h->G_sp, h->G_s, h->rec, nullptr,
                                                          h->Gv, nullptr);
  LAUNCHCHK();
  // dense inverse of the top block for the batched solves: the top solve
  // applied to the identity, then its transpose
  if (P.ntop > 0 && (size_t)P.ntop * 2 * sizeof(double) <= 64 * 1024) {
    const int nt = P.ntop;
    k_identity_block<<<dim3(cdiv(nt, 64), cdiv(nt, 4)), dim3(64, 4), 0, s>>>(nt, nt, 0, h->top_inv, nt);
    LAUNCHCHK();
    const int twt = h->tw_top;
    k_top_dense<<<cdiv(nt, twt), 256, (size_t)nt * twt * sizeof(double), s>>>(0, nt, h->dense_top, h->top_dinv,
                                                                             h->top_inv, nt, nt, twt, nullptr);
    LAUNCHCHK();
    k_transpose<<<dim3(cdiv(nt, 32), cdiv(nt, 32)), dim3(32, 8), 0, s>>>(nt, h->top_inv, h->top_invT, nullptr);
    LAUNCHCHK();
    h->top_inv_ok = true;
  }
  h->rho = rho;
  h->have_point = true;
}


// H and/or J (row-major, n_u columns) from batches of identity directions at
// the cached point; batch 0 = the handle's width.  Batches run on the
// handle's streams (forked from s, joined back) unless s is being captured.
void derivative_batches(rpf_grid* h, double* H, double* J, int batch, hipStream_t s) {
  const int nu = h->P.nu;
  const int B = batch == 0 ? std::min(h->max_batch, nu) : std::min<int>(batch, std::min(h->max_batch, nu));
  const int nbt = cdiv(nu, B);
  // one stream while `s` is being captured into a graph: the fork onto the
  // handle's streams is not used under capture
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(s, &cap));
  const int nst = cap == hipStreamCaptureStatusNone ? std::min(h->nhs, nbt) : 1;
  if (nst <= 1) {
    for (int j0 = 0; j0 < nu; j0 += B)
      hvp_batch(h, nullptr, 0, j0, std::min(B, nu - j0), H ? H + j0 : nullptr, nu, s, 0, J, nu);
  } else {
    // fork: batch b on internal stream b % nst with its own workspace;
    // join back on the caller's stream
    HIPCHK(hipEventRecord(h->ev_fork, s));
    for (int k = 0; k < nst; ++k) HIPCHK(hipStreamWaitEvent(h->hs[k], h->ev_fork, 0));
    for (int b = 0; b < nbt; ++b) {
      const int j0 = b * B;
      hvp_batch(h, nullptr, 0, j0, std::min(B, nu - j0), H ? H + j0 : nullptr, nu, h->hs[b % nst], b % nst, J, nu);
    }
    for (int k = 0; k < nst; ++k) {
      HIPCHK(hipEventRecord(h->ev_join[k], h->hs[k]));
      HIPCHK(hipStreamWaitEvent(s, h->ev_join[k], 0));
    }
  }
}

// Second-order data of the cached point (bus weights with lambda, branch
// 4x4 blocks, K and its diagonal terms, rank-one coefficients) rebuilt with
// the constraints' curvature weights gn [m] in place of rho sigma_k^2 (gn
// null: the point's own weights).
void second_order(rpf_grid* h, const ALArgs& A, const VarArgs& V, const double* gn, const double* sigma, double rho,
                  hipStream_t s, const int32_t* skip) {
  const Presolve& P = h->P;
  const int nbw = cdiv(P.nb + 2 + P.npv, 256);
  k_bus_weights<<<nbw, 256, 0, s>>>(A, h->wvec, h->lam, h->rowP, h->rowQ, h->bus_pvpos, h->a, h->b, h->kappa, gn,
                                    skip);
  LAUNCHCHK();
  k_branch_second<<<cdiv(P.nl, 256), 256, 0, s>>>(P.nl, h->br_f, h->br_t, h->br_r, h->br_x, h->br_b, h->th, h->vm,
                                                   h->rec, h->a, h->b, h->wvec, sigma + 1, rho, h->wrec, gn, skip);
  LAUNCHCHK();
  k_gather_sum<<<cdiv(P.K_col.size(), 256), 256, 0, s>>>((int)P.K_col.size(), h->K_sp, h->K_s, h->wrec, nullptr,
                                                          h->Kv, skip);
  LAUNCHCHK();
  k_k_diag<<<cdiv(P.nvar, 256), 256, 0, s>>>(V, h->K_diag, sigma + 1, rho, h->Kv, gn, skip);
  LAUNCHCHK();
}

// out = alpha A^T x + beta b (b may be null) for a row-major rows x cols A:
// partial sums over qparts row chunks, then their sum in chunk order.
void gemv_t(rpf_grid* h, const double* A, int rows, int cols, const double* x, double alpha, const double* b,
            double beta, double* out, hipStream_t s, const int32_t* skip) {
  const int R = h->qparts;
  const int chunk = cdiv(rows, R);
  k_gemv_cols_part<<<dim3(cdiv(cols, 256), R), 256, 0, s>>>(rows, cols, chunk, A, cols, x, h->qpart, skip);
  LAUNCHCHK();
  k_gemv_cols_sum<<<cdiv(cols, 256), 256, 0, s>>>(cols, R, h->qpart, alpha, b, beta, out, skip);
  LAUNCHCHK();
}

QPVec qp_vec(rpf_grid* h, double rho, double delta, double tol, const double* sigma) {
  QPVec Q;
  Q.nu = h->P.nu; Q.m = h->P.m; Q.rho = rho; Q.delta = delta; Q.tol = tol;
  Q.sigma_c = sigma + 1;
  Q.g = h->qg; Q.d = h->qd_; Q.tl = h->qtl; Q.tu = h->qtu; Q.zl = h->qzl; Q.zu = h->qzu; Q.sig = h->qsig;
  Q.cs = h->qcs; Q.gn = h->qgn; Q.base = h->qbase; Q.dda = h->qdda; Q.dzla = h->qdzla; Q.dzua = h->qdzua;
  Q.rhs = h->qrhs; Q.dd = h->qdd; Q.dzl = h->qdzl; Q.dzu = h->qdzu; Q.ts = h->qts; Q.rneg = h->qrneg;
  Q.xu = h->qxu; Q.Hd = h->qHd; Q.Jv = h->qJv; Q.Jt = h->qJt; Q.qs = h->qscal;
  Q.done = h->qflags + QF_DONE; Q.iters = h->qflags + QF_ITERS; Q.retry = h->qflags + QF_RETRY;
  Q.skF = h->qflags + QF_SKF; Q.sk2 = h->qflags + QF_SK2; Q.cinfo = h->qflags + QF_CINFO;
  Q.fact = h->qflags + QF_FACT;
  return Q;
}

// Schur solve of (Hw + Sigma + w P_u) x = b (Proposition 3) with S + w I
// factorized in Sf: xu = (S + w I)^{-1} (b_u + rho J^T ts), Jv = J xu
// (ts = sigma^2 b_s / C is already in Q.ts); the s part is formed by the
// next vector step.  Skipped while sk2 is set.
void qp_schur_solve(rpf_grid* h, const QPVec& Q, const double* J, const double* Sf, const double* b, hipStream_t s) {
  const int nu = Q.nu, m = Q.m;
  gemv_t(h, J, m, nu, Q.ts, -Q.rho, b, -1.0, Q.rneg, s, Q.sk2);
  // chol_solve gives -S^{-1} rneg; its kernels return at once while sk2 != 0
  // (and a solve that gives up waiting writes -1 there)
  chol_solve(h, nu, Sf, Q.rneg, Q.xu, Q.sk2, s);
  k_gemv_rows<<<cdiv(m, 4), 256, 0, s>>>(m, nu, J, nu, Q.xu, Q.Jv, Q.sk2);
  LAUNCHCHK();
}

// Hw d pieces for the KKT test: Hd = H d_u, Jv = J d_u, Jt = J^T ts.
void qp_kkt_products(rpf_grid* h, const QPVec& Q, const double* H, const double* J, hipStream_t s) {
  const int nu = Q.nu, m = Q.m;
  k_gemv_rows<<<cdiv(nu, 4), 256, 0, s>>>(nu, nu, H, nu, Q.d, Q.Hd, Q.skF);
  LAUNCHCHK();
  k_gemv_rows<<<cdiv(m, 4), 256, 0, s>>>(m, nu, J, nu, Q.d, Q.Jv, Q.skF);
  LAUNCHCHK();
  gemv_t(h, J, m, nu, Q.ts, 1.0, nullptr, 0.0, Q.Jt, s, Q.skF);
}

// The bounded QP at the cached point (rpf_qp_step after its derivatives):
// max_iter predicated slots (an iteration, or a retried factorization with
// a larger regularisation), then a last KKT test.
void qp_ipm(rpf_grid* h, const ALArgs& A, const VarArgs& V, const double* H, const double* J, double* Sf,
            const double* u, const double* sv, const double* u_lo, const double* u_hi, const double* s_lo,
            const double* s_hi, double rho, const double* sigma, double delta, int max_iter, double tol, int batch,
            hipStream_t s) {
  const int nu = h->P.nu;
  const QPVec Q = qp_vec(h, rho, delta, tol, sigma);
  double* S = h->qS;
  k_qp_init<<<1, QP_NT, 0, s>>>(Q, u, sv, u_lo, u_hi, s_lo, s_hi, h->gradbuf, h->wvec, H);
  LAUNCHCHK();
  for (int it = 0; it <= max_iter; ++it) {
    k_qp_slot<<<1, 64, 0, s>>>(Q);
    LAUNCHCHK();
    qp_kkt_products(h, Q, H, J, s);
    k_qp_kkt<<<1, QP_NT, 0, s>>>(Q, it == max_iter ? 1 : 0);
    LAUNCHCHK();
    if (it == max_iter) break;
    // S = H_gn + Sigma_u + delta I: the reduced Hessian with the Schur
    // curvature weights, by the batched products (skipped on a retry)
    h->skipw = Q.skF;
    try {
      second_order(h, A, V, Q.gn, sigma, rho, s, Q.skF);
      derivative_batches(h, S, nullptr, batch, s);
    } catch (...) {
      h->skipw = nullptr;
      throw;
    }
    h->skipw = nullptr;
    k_symmetrize<<<dim3(cdiv(nu, 32), cdiv(nu, 32)), dim3(32, 8), 0, s>>>(nu, S, Q.sig, delta, Q.skF);
    LAUNCHCHK();
    // inertia control: Cholesky of S + w I
    k_qp_reg_set<<<1, 64, 0, s>>>(Q);
    LAUNCHCHK();
    k_qp_reg_copy<<<cdiv((long)nu * nu, 256), 256, 0, s>>>(nu, S, Sf, Q);
    LAUNCHCHK();
    dense_factor<true>(nu, Sf, Q.cinfo, 0, s);
    k_qp_reg_check<<<1, 64, 0, s>>>(Q);
    LAUNCHCHK();
    // predictor, then corrector with the same factor
    qp_schur_solve(h, Q, J, Sf, Q.base, s);
    k_qp_pred<<<1, QP_NT, 0, s>>>(Q);
    LAUNCHCHK();
    qp_schur_solve(h, Q, J, Sf, Q.rhs, s);
    k_qp_corr<<<1, QP_NT, 0, s>>>(Q);
    LAUNCHCHK();
  }
  // the point's own second-order data back for later Hessian products
  second_order(h, A, V, nullptr, sigma, rho, s, nullptr);
}

}  // namespace

extern "C" {

int rpf_reduced_gradient(rpf_grid* h, const double* x, const double* u, const double* pd, const double* qd,
                         const double* sv, const double* y, double rho, const double* sigma, double* grad,
                         double* lambda, int32_t* info, rpf_stream_t stream) {
  if (!h || !x || !u || !pd || !qd || !sv || !y || !sigma || !grad) return set_err(RPF_EINVAL, "NULL argument");
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    Traced trace_scope(h, "rpf_reduced_gradient", s);
    x_in(h, x, s);
    gradient_core(h, u, pd, qd, sv, y, rho, sigma, grad, lambda, s);
    if (info) {
      k_piv_report<<<1, 1, 0, s>>>(h->piv_status, h->x_i2p, info);
      LAUNCHCHK();
    }
    return RPF_OK;
  });
}

int rpf_reduced_hessian_batch(rpf_grid* h, const double* V, int32_t nbatch, int32_t ldv, double* HV,
                              int32_t ldhv, rpf_stream_t stream) {
  if (!h || !V || !HV) return set_err(RPF_EINVAL, "NULL argument");
  if (!h->have_point) return set_err(RPF_ESTATE, "no cached point: call rpf_reduced_gradient first");
  if (nbatch < 1 || nbatch > h->max_batch) return set_err(RPF_ESIZE, "nbatch outside [1, max_batch]");
  if (ldv < nbatch || ldhv < nbatch) return set_err(RPF_EINVAL, "leading dimension below nbatch");
  return guard([&]() -> int {
    Traced trace_scope(h, "rpf_reduced_hessian_batch", (hipStream_t)stream, (long long)nbatch);
    hvp_batch(h, V, ldv, 0, nbatch, HV, ldhv, (hipStream_t)stream);
    return RPF_OK;
  });
}

int rpf_reduced_derivatives(rpf_grid* h, double* H, double* J, int32_t batch, rpf_stream_t stream) {
  if (!h || (!H && !J)) return set_err(RPF_EINVAL, "NULL argument: H and J are both NULL (or no grid)");
  if (!h->have_point) return set_err(RPF_ESTATE, "no cached point: call rpf_reduced_gradient first");
  if (batch < 0) return set_err(RPF_EINVAL, "batch must be >= 0");
  return guard([&]() -> int {
    Traced trace_scope(h, "rpf_reduced_derivatives", (hipStream_t)stream, (long long)batch);
    derivative_batches(h, H, J, batch, (hipStream_t)stream);
    return RPF_OK;
  });
}

int rpf_reduced_hessian(rpf_grid* h, double* H, int32_t batch, rpf_stream_t stream) {
  if (!h || !H) return set_err(RPF_EINVAL, "NULL argument");
  return rpf_reduced_derivatives(h, H, nullptr, batch, stream);
}

int rpf_factor_solve(rpf_grid* h, int32_t n, double* K, const double* diag, double delta, const double* rhs,
                     double* step, int32_t* info, rpf_stream_t stream) {
  if (!h || !K || !rhs || !step || !info) return set_err(RPF_EINVAL, "NULL argument");
  if (n < 1 || n > h->P.nu) return set_err(RPF_EINVAL, "n must be in [1, n_u]");
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    Traced trace_scope(h, "rpf_factor_solve", s, (long long)n);
    size_t pi = h->prof_on ? h->prof_begin(s) : 0;
    factor_solve_ws(n, K, diag, delta, rhs, step, info, h->chol_flags, h->chol_dinv, h->chol_work, s);
    if (h->prof_on) h->prof_end(4, pi, s);
    return RPF_OK;
  });
}

int rpf_qp_step(rpf_grid* h, const double* x, const double* u, const double* pd, const double* qd, const double* sv,
                const double* y, double rho, const double* sigma, double delta, const double* u_lo,
                const double* u_hi, const double* s_lo, const double* s_hi, int32_t max_iter, double tol,
                int32_t batch, double* H, double* J, double* grad, double* dw, double* zw, double* kkt,
                double* wreg, int32_t* status, rpf_stream_t stream) {
  if (!h || !x || !u || !pd || !qd || !sv || !y || !sigma || !u_lo || !u_hi || !s_lo || !s_hi || !J || !dw ||
      !status)
    return set_err(RPF_EINVAL, "NULL argument");
  if (max_iter < 0 || max_iter > 500) return set_err(RPF_EINVAL, "max_iter must be in [0, 500]");
  if (batch < 0) return set_err(RPF_EINVAL, "batch must be >= 0");
  if (!(rho > 0.0)) return set_err(RPF_EINVAL, "rho must be positive");
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    Traced trace_scope(h, "rpf_qp_step", s, (long long)max_iter);
    const Presolve& P = h->P;
    const int nu = P.nu, n = P.nu + P.m;
    double* Hm = H ? H : h->Hbuf;
    // 1. point: power-flow state x, reduced gradient, cached second-order data
    x_in(h, x, s);
    gradient_core(h, u, pd, qd, sv, y, rho, sigma, h->gradbuf, nullptr, s);
    k_piv_report<<<1, 1, 0, s>>>(h->piv_status, h->x_i2p, h->qflags + QF_PIV);
    LAUNCHCHK();
    // 2. reduced Hessian and Jacobian from the same identity batches,
    // H symmetrised
    derivative_batches(h, Hm, J, batch, s);
    k_symmetrize<<<dim3(cdiv(nu, 32), cdiv(nu, 32)), dim3(32, 8), 0, s>>>(nu, Hm, nullptr, 0.0);
    LAUNCHCHK();
    // 3. the QP
    const ALArgs A = al_args(h, u, pd, qd, sv, y, rho, sigma);
    const VarArgs V = var_args(h, u, sigma);
    qp_ipm(h, A, V, Hm, J, h->Kbuf, u, sv, u_lo, u_hi, s_lo, s_hi, rho, sigma, delta, max_iter, tol, batch, s);
    k_copy_vec<<<cdiv(n, 256), 256, 0, s>>>(n, h->qd_, dw, nullptr);
    LAUNCHCHK();
    if (zw) {
      k_copy_vec<<<cdiv(n, 256), 256, 0, s>>>(n, h->qzl, zw, nullptr);
      LAUNCHCHK();
      k_copy_vec<<<cdiv(n, 256), 256, 0, s>>>(n, h->qzu, zw + n, nullptr);
      LAUNCHCHK();
    }
    if (grad) {
      k_copy_vec<<<cdiv(nu, 256), 256, 0, s>>>(nu, h->gradbuf, grad, nullptr);
      LAUNCHCHK();
    }
    k_qp_status<<<1, 1, 0, s>>>(h->qflags, h->qscal, status, kkt, wreg);
    LAUNCHCHK();
    return RPF_OK;
  });
}

int rpf_track_step(rpf_grid* h, double* u, double* x, double* y, const double* pd0, const double* qd0,
                   const double* load_factor, const double* s_lo, const double* s_hi, const double* u_lo,
                   const double* u_hi, double rho, const double* sigma, double delta, int32_t pf_iters,
                   int32_t max_halvings, double tol, int32_t* status, rpf_stream_t stream) {
  if (!h || !u || !x || !y || !pd0 || !qd0 || !load_factor || !s_lo || !s_hi || !u_lo || !u_hi || !sigma || !status)
    return set_err(RPF_EINVAL, "NULL argument");
  if (pf_iters < 1 || max_halvings < 0 || max_halvings > 30) return set_err(RPF_EINVAL, "bad iteration counts");
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    Traced trace_scope(h, "rpf_track_step", s);
    const Presolve& P = h->P;
    const int nu = P.nu, nx = P.nx, m = P.m;
    int32_t* done = h->tflags;        // predication flag of the current power flow
    int32_t* count = h->tflags + 1;
    int32_t* accepted = h->tflags + 2;
    int32_t* which = h->tflags + 3;
    int32_t* info = h->tflags + 4;
    k_fill_int<<<1, 8, 0, s>>>(8, h->tflags, 0);
    LAUNCHCHK();
    k_fill_int<<<1, 1, 0, s>>>(1, which, -1);
    LAUNCHCHK();
    k_track_loads<<<cdiv(P.nb, 256), 256, 0, s>>>(P.nb, pd0, qd0, load_factor, h->pdt, h->qdt);
    LAUNCHCHK();
    // 1. power flow at the current control and the new loads (warm start)
    x_in(h, x, s);
    pf_device(h, u, h->pdt, h->qdt, pf_iters, tol, done, count, h->tres, s);
    k_copy_int<<<1, 1, 0, s>>>(done, h->tflags + 5);
    LAUNCHCHK();
    k_copy_int<<<1, 1, 0, s>>>(count, h->tflags + 6);
    LAUNCHCHK();
    // 2. slack minimiser at the current multipliers
    state_and_records(h, u, s);
    bus_injections(h, s);
    ALArgs A = al_args(h, u, h->pdt, h->qdt, h->scur, y, rho, sigma);
    k_constraints<<<cdiv(m + P.ng, 256), 256, 0, s>>>(A, h->cvec, nullptr, nullptr);
    LAUNCHCHK();
    k_slack<<<cdiv(m, 256), 256, 0, s>>>(m, h->cvec, y, sigma + 1, rho, s_lo, s_hi, h->scur);
    LAUNCHCHK();
    // 3. reduced gradient and Hessian at (u, s, y)
    gradient_core(h, u, h->pdt, h->qdt, h->scur, y, rho, sigma, h->gradbuf, nullptr, s);
    k_piv_report<<<1, 1, 0, s>>>(h->piv_status, h->x_i2p, h->tflags + 7);
    LAUNCHCHK();
    const int B = std::min(h->max_batch, nu);
    for (int j0 = 0; j0 < nu; j0 += B) hvp_batch(h, nullptr, 0, j0, std::min(B, nu - j0), h->Hbuf + j0, nu, s);
    // 4. step = -(H + delta I)^{-1} grad (zero when the factorization fails)
    k_copy_vec<<<cdiv((long)nu * nu, 256), 256, 0, s>>>(nu * nu, h->Hbuf, h->Kbuf, nullptr);
    LAUNCHCHK();
    k_symmetrize<<<dim3(cdiv(nu, 32), cdiv(nu, 32)), dim3(32, 8), 0, s>>>(nu, h->Kbuf, nullptr, delta);
    LAUNCHCHK();
    factor_then_solve(nu, h->Kbuf, h->gradbuf, h->dstep, info, h->chol_flags, h->chol_dinv, h->chol_work, s);
    k_zero_if<<<cdiv(nu, 256), 256, 0, s>>>(nu, info, h->dstep);
    LAUNCHCHK();
    // 5. u + step / 2^k clipped to the bounds, first k whose power flow converges
    k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi, h->xi_save, nullptr);
    LAUNCHCHK();
    double f = 1.0;
    for (int k = 0; k <= max_halvings; ++k, f *= 0.5) {
      k_try_u<<<cdiv(nu, 256), 256, 0, s>>>(nu, u, h->dstep, f, u_lo, u_hi, h->u_try, accepted);
      LAUNCHCHK();
      k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi_save, h->xi, accepted);
      LAUNCHCHK();
      k_copy_int<<<1, 1, 0, s>>>(accepted, done);
      LAUNCHCHK();
      pf_device(h, h->u_try, h->pdt, h->qdt, pf_iters, tol, done, count, h->tres + 1, s);
      k_accept<<<1, 256, 0, s>>>(nu, h->tres + 1, tol, accepted, h->u_try, u, k, which);
      LAUNCHCHK();
    }
    // no trial accepted: keep u and the power flow at u
    k_fill_int<<<1, 1, 0, s>>>(1, done, 0);
    LAUNCHCHK();
    k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi_save, h->xi, accepted);
    LAUNCHCHK();
    // 6. constraints at the new point, slack minimiser and multiplier update
    state_and_records(h, u, s);
    bus_injections(h, s);
    k_constraints<<<cdiv(m + P.ng, 256), 256, 0, s>>>(A, h->cvec, nullptr, nullptr);
    LAUNCHCHK();
    k_y_update<<<cdiv(m, 256), 256, 0, s>>>(m, h->cvec, sigma + 1, rho, s_lo, s_hi, y, h->scur);
    LAUNCHCHK();
    k_permute_scatter<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->x_i2p, h->xi, x, nullptr);
    LAUNCHCHK();
    k_track_status<<<1, 1, 0, s>>>(h->tflags, status);
    LAUNCHCHK();
    return RPF_OK;
  });
}


int rpf_track_step_qp(rpf_grid* h, double* u, double* sv, double* x, double* y, const double* pd0,
                      const double* qd0, const double* load_factor, const double* s_lo, const double* s_hi,
                      const double* u_lo, const double* u_hi, double rho, const double* sigma, double delta,
                      int32_t pf_iters, int32_t max_halvings, double tol, int32_t qp_iters, double qp_tol,
                      int32_t batch, double dispatch_scale, double* J, int32_t* status, rpf_stream_t stream) {
  if (!h || !u || !sv || !x || !y || !pd0 || !qd0 || !load_factor || !s_lo || !s_hi || !u_lo || !u_hi || !sigma ||
      !J || !status)
    return set_err(RPF_EINVAL, "NULL argument");
  if (pf_iters < 1 || max_halvings < 0 || max_halvings > 30 || qp_iters < 0 || qp_iters > 500)
    return set_err(RPF_EINVAL, "bad iteration counts");
  if (batch < 0) return set_err(RPF_EINVAL, "batch must be >= 0");
  if (!(rho > 0.0)) return set_err(RPF_EINVAL, "rho must be positive");
  if (!(dispatch_scale > 0.0)) return set_err(RPF_EINVAL, "dispatch_scale must be positive");
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    Traced trace_scope(h, "rpf_track_step_qp", s);
    const Presolve& P = h->P;
    const int nu = P.nu, nx = P.nx, m = P.m;
    int32_t* done = h->tflags;        // predication flag of the current power flow
    int32_t* count = h->tflags + 1;
    int32_t* accepted = h->tflags + 2;
    int32_t* which = h->tflags + 3;
    k_fill_int<<<1, 8, 0, s>>>(8, h->tflags, 0);
    LAUNCHCHK();
    k_fill_int<<<1, 1, 0, s>>>(1, which, -1);
    LAUNCHCHK();
    k_track_loads<<<cdiv(P.nb, 256), 256, 0, s>>>(P.nb, pd0, qd0, load_factor, h->pdt, h->qdt);
    LAUNCHCHK();
    if (dispatch_scale != 1.0 && P.npv > 0) {
      // p_pv, the last n_pv controls, follow a uniform load change
      k_scale_vec<<<cdiv(P.npv, 256), 256, 0, s>>>(P.npv, dispatch_scale, u + 1 + P.npv);
      LAUNCHCHK();
    }
    // 1. power flow at the current control and the new loads (warm start)
    x_in(h, x, s);
    pf_device(h, u, h->pdt, h->qdt, pf_iters, tol, done, count, h->tres, s);
    k_copy_int<<<1, 1, 0, s>>>(done, h->tflags + 5);
    LAUNCHCHK();
    k_copy_int<<<1, 1, 0, s>>>(count, h->tflags + 6);
    LAUNCHCHK();
    // 2. the bounded QP at (u, s, y): gradient, H and J, interior point
    gradient_core(h, u, h->pdt, h->qdt, sv, y, rho, sigma, h->gradbuf, nullptr, s);
    k_piv_report<<<1, 1, 0, s>>>(h->piv_status, h->x_i2p, h->tflags + 7);
    LAUNCHCHK();
    derivative_batches(h, h->Hbuf, J, batch, s);
    k_symmetrize<<<dim3(cdiv(nu, 32), cdiv(nu, 32)), dim3(32, 8), 0, s>>>(nu, h->Hbuf, nullptr, 0.0);
    LAUNCHCHK();
    {
      const ALArgs A = al_args(h, u, h->pdt, h->qdt, sv, y, rho, sigma);
      const VarArgs V = var_args(h, u, sigma);
      qp_ipm(h, A, V, h->Hbuf, J, h->Kbuf, u, sv, u_lo, u_hi, s_lo, s_hi, rho, sigma, delta, qp_iters, qp_tol,
             batch, s);
    }
    // 3. w + dw / 2^k for the first k whose power flow converges
    k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi, h->xi_save, nullptr);
    LAUNCHCHK();
    double f = 1.0;
    for (int k = 0; k <= max_halvings; ++k, f *= 0.5) {
      k_try_w<<<cdiv(nu + m, 256), 256, 0, s>>>(nu, m, u, sv, h->qd_, f, h->u_try, h->s_try, accepted);
      LAUNCHCHK();
      k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi_save, h->xi, accepted);
      LAUNCHCHK();
      k_copy_int<<<1, 1, 0, s>>>(accepted, done);
      LAUNCHCHK();
      pf_device(h, h->u_try, h->pdt, h->qdt, pf_iters, tol, done, count, h->tres + 1, s);
      k_accept_w<<<1, 256, 0, s>>>(nu, m, h->tres + 1, tol, accepted, h->u_try, h->s_try, u, sv, k, which);
      LAUNCHCHK();
    }
    // no trial accepted: keep (u, s) and the power flow at u
    k_fill_int<<<1, 1, 0, s>>>(1, done, 0);
    LAUNCHCHK();
    k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi_save, h->xi, accepted);
    LAUNCHCHK();
    // 4. multiplier update at the new point: y += rho D_c (c(u) - s)
    state_and_records(h, u, s);
    bus_injections(h, s);
    const ALArgs A2 = al_args(h, u, h->pdt, h->qdt, sv, y, rho, sigma);
    k_constraints<<<cdiv(m + P.ng, 256), 256, 0, s>>>(A2, h->cvec, nullptr, nullptr);
    LAUNCHCHK();
    k_y_update_s<<<cdiv(m, 256), 256, 0, s>>>(m, h->cvec, sigma + 1, rho, sv, y);
    LAUNCHCHK();
    k_permute_scatter<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->x_i2p, h->xi, x, nullptr);
    LAUNCHCHK();
    k_track_qp_status<<<1, 1, 0, s>>>(h->tflags, h->qflags, status);
    LAUNCHCHK();
    return RPF_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------- static OPF
namespace {

// AL value (and, with cost, the cost f times sigma_f) at the state in h->xi,
// control u, slack sv; c into h->cvec.  Device scalars out.
void al_value(rpf_grid* h, const double* u, const double* pd, const double* qd, const double* sv, const double* y,
              double rho, const double* sigma, double* phi, double* cost, hipStream_t s) {
  const Presolve& P = h->P;
  state_and_records(h, u, s);
  bus_injections(h, s);
  ALArgs A = al_args(h, u, pd, qd, sv, y, rho, sigma);
  k_constraints<<<cdiv(P.m + P.ng, 256), 256, 0, s>>>(A, h->cvec, nullptr, h->terms);
  LAUNCHCHK();
  k_reduce_final<<<1, 1024, 0, s>>>(P.m + P.ng, h->terms, phi, 0, 0.0, nullptr, nullptr);
  LAUNCHCHK();
  if (cost) {
    k_reduce_final<<<1, 1024, 0, s>>>(P.ng, h->terms + P.m, cost, 0, 0.0, nullptr, nullptr);
    LAUNCHCHK();
  }
}

template <class T>
T read1(const T* d, hipStream_t s) {
  T v;
  HIPCHK(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return v;
}

}  // namespace

extern "C" {

int rpf_static_opf(rpf_grid* h, double* x, double* u, double* sv, double* y, const double* pd, const double* qd,
                   double rho0, const double* sigma, const double* u_lo, const double* u_hi, const double* s_lo,
                   const double* s_hi, int32_t max_outer, int32_t max_inner, int32_t qp_iters, double qp_tol,
                   int32_t pf_iters, double tol, double* J, double* hist, int32_t* nhist, double* rho_out,
                   rpf_stream_t stream) {
  if (!h || !x || !u || !sv || !y || !pd || !qd || !sigma || !u_lo || !u_hi || !s_lo || !s_hi || !J || !hist ||
      !nhist)
    return set_err(RPF_EINVAL, "NULL argument");
  if (!(rho0 > 0.0)) return set_err(RPF_EINVAL, "rho must be positive");
  if (max_outer < 1 || max_outer > 1000 || max_inner < 0 || max_inner > 1000 || qp_iters < 1 || qp_iters > 500 ||
      pf_iters < 1 || pf_iters > 100)
    return set_err(RPF_EINVAL, "bad iteration counts");
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    Traced trace_scope(h, "rpf_static_opf", s, (long long)max_outer);
    const Presolve& P = h->P;
    const int nu = P.nu, nx = P.nx, m = P.m;
    const double kArmijo = 1e-4, kRhoUp = 10.0, kEtaPrimal = 1e-5, kEtaDual = 1e-4;
    const int kHalvings = 10;
    double* sc = h->resid_d;   // device scalars: [0] pg, [1] slope, [2] phi, [3] cost
    double* sc2 = h->tres;     // [0] theta, [1] trial phi
    int32_t* done = h->flag;
    int32_t* count = h->flag + 1;
    *nhist = 0;
    // the state at the starting control
    x_in(h, x, s);
    k_fill_int<<<1, 4, 0, s>>>(4, h->flag, 0);
    LAUNCHCHK();
    pf_device(h, u, pd, qd, pf_iters, tol, done, count, sc2, s);
    if (read1(done, s) != 1) return set_err(RPF_EINVAL, "power flow at the starting control did not converge");
    const double sigf = read1(sigma, s);
    double rho = rho0, omega = 1.0 / rho0, eta = 1.0 / std::pow(rho0, 0.1);
    for (int k = 0; k < max_outer; ++k) {
      int inner = 0;
      double pg = 0.0;
      for (inner = 0; inner <= max_inner; ++inner) {
        // the bounded QP of L_rho at (u, s, y): gradient, H, J, interior point
        gradient_core(h, u, pd, qd, sv, y, rho, sigma, h->gradbuf, nullptr, s);
        derivative_batches(h, h->Hbuf, J, 0, s);
        k_symmetrize<<<dim3(cdiv(nu, 32), cdiv(nu, 32)), dim3(32, 8), 0, s>>>(nu, h->Hbuf, nullptr, 0.0);
        LAUNCHCHK();
        {
          const ALArgs A = al_args(h, u, pd, qd, sv, y, rho, sigma);
          const VarArgs V = var_args(h, u, sigma);
          qp_ipm(h, A, V, h->Hbuf, J, h->Kbuf, u, sv, u_lo, u_hi, s_lo, s_hi, rho, sigma, 0.0, qp_iters, qp_tol, 0,
                 s);
        }
        k_static_pg<<<1, QP_NT, 0, s>>>(nu, m, u, sv, u_lo, u_hi, s_lo, s_hi, h->qg, h->qd_, sc);
        LAUNCHCHK();
        double pv[2];
        HIPCHK(hipMemcpyAsync(pv, sc, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        pg = pv[0];
        const double slope = pv[1];
        if (pg <= omega || inner == max_inner) break;
        if (!(slope < 0.0)) break;
        // backtracking line search on L_rho, a power flow at each trial point
        al_value(h, u, pd, qd, sv, y, rho, sigma, sc + 2, nullptr, s);
        const double phi0 = read1(sc + 2, s);
        k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi, h->xi_save, nullptr);
        LAUNCHCHK();
        bool accepted = false;
        double a = 1.0;
        for (int hh = 0; hh <= kHalvings; ++hh, a *= 0.5) {
          k_try_w<<<cdiv(nu + m, 256), 256, 0, s>>>(nu, m, u, sv, h->qd_, a, h->u_try, h->s_try, nullptr);
          LAUNCHCHK();
          k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi_save, h->xi, nullptr);
          LAUNCHCHK();
          k_fill_int<<<1, 4, 0, s>>>(4, h->flag, 0);
          LAUNCHCHK();
          pf_device(h, h->u_try, pd, qd, pf_iters, tol, done, count, sc2, s);
          if (read1(done, s) != 1) continue;
          al_value(h, h->u_try, pd, qd, h->s_try, y, rho, sigma, sc2 + 1, nullptr, s);
          const double phi = read1(sc2 + 1, s);
          if (phi <= phi0 + kArmijo * a * slope) {
            k_copy_vec<<<cdiv(nu, 256), 256, 0, s>>>(nu, h->u_try, u, nullptr);
            LAUNCHCHK();
            k_copy_vec<<<cdiv(m, 256), 256, 0, s>>>(m, h->s_try, sv, nullptr);
            LAUNCHCHK();
            accepted = true;
            break;
          }
        }
        if (!accepted) {
          k_copy_vec<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->xi_save, h->xi, nullptr);
          LAUNCHCHK();
          break;
        }
      }
      // primal infeasibility, multipliers or penalty
      al_value(h, u, pd, qd, sv, y, rho, sigma, sc + 2, sc + 3, s);
      k_static_theta<<<1, QP_NT, 0, s>>>(m, h->cvec, sv, sc2);
      LAUNCHCHK();
      const double theta = read1(sc2, s);
      const double fcost = read1(sc + 3, s) / sigf;
      double* rec = hist + (size_t)k * 8;
      rec[0] = rho; rec[1] = inner; rec[2] = theta; rec[3] = pg; rec[4] = fcost; rec[5] = 0.0; rec[6] = 0.0;
      rec[7] = read1(sc + 2, s);
      *nhist = k + 1;
      if (theta <= eta) {
        if (theta <= kEtaPrimal && pg <= kEtaDual) {
          rec[6] = 1.0;
          break;
        }
        k_y_update_s<<<cdiv(m, 256), 256, 0, s>>>(m, h->cvec, sigma + 1, rho, sv, y);
        LAUNCHCHK();
        eta /= std::pow(rho, 0.9);
        omega /= rho;
        rec[5] = 1.0;
      } else {
        rho *= kRhoUp;
        eta = 1.0 / std::pow(rho, 0.1);
        omega = 1.0 / rho;
      }
    }
    if (rho_out) *rho_out = rho;
    k_permute_scatter<<<cdiv(nx, 256), 256, 0, s>>>(nx, h->x_i2p, h->xi, x, nullptr);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));
    h->have_point = false;
    return RPF_OK;
  });
}

}  // extern "C"

// ------------------------------------------------- no-allocation dense step
// Scratch of rpf_factor_solve_noalloc in a static device array (one copy per
// GPU, held until the process ends): the inverses of the diagonal blocks
// [cdiv(n, CB) 2 CB CB], the forward-solve vector [n] and the block flags
// [2 cdiv(n, CB)] int32, for n <= RPF_NOALLOC_MAX_N.
namespace {
constexpr int kNoallocBlocks = RPF_NOALLOC_MAX_N / CB;
constexpr size_t kNoallocDinv = (size_t)kNoallocBlocks * 2 * CB * CB;
constexpr size_t kNoallocWork = RPF_NOALLOC_MAX_N;
constexpr size_t kNoallocFlags = 2 * kNoallocBlocks;   // int32 words
constexpr size_t kNoallocDoubles = kNoallocDinv + kNoallocWork + (kNoallocFlags + 1) / 2;
static_assert(RPF_NOALLOC_MAX_N % CB == 0, "maximum order must be a multiple of the block width");
}  // namespace

static __device__ __align__(256) double scratch[kNoallocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device, looked up once per
// device (the array's host-side name is not a device address)
double* noalloc_scratch() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw std::runtime_error("device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw HipError("hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_ptr[dev] = (double*)p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int rpf_factor_solve_noalloc(int32_t n, double* K, const double* diag, double delta, const double* rhs,
                                        double* step, int32_t* info, rpf_stream_t stream) {
  if (!K || !rhs || !step || !info) return set_err(RPF_EINVAL, "NULL argument");
  if (n < 1) return set_err(RPF_EINVAL, "n must be >= 1");
  if (n > RPF_NOALLOC_MAX_N)
    return set_err(RPF_ESIZE, "n = " + std::to_string(n) + " above the scratch limit RPF_NOALLOC_MAX_N = " +
                                  std::to_string(RPF_NOALLOC_MAX_N));
  return guard([&]() -> int {
    double* base = noalloc_scratch();
    double* dinv = base;
    double* work = base + kNoallocDinv;
    int32_t* flags = reinterpret_cast<int32_t*>(work + kNoallocWork);
    factor_solve_ws(n, K, diag, delta, rhs, step, info, flags, dinv, work, (hipStream_t)stream);
    return RPF_OK;
  });
}
