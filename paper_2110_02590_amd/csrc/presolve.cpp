// Host presolve: index maps, ordering, symbolic LU, level sets and gather
// lists.  Pure integer work, run once per topology.
#include "presolve.hpp"

#include <algorithm>
#include <map>
#include <numeric>
#include <set>
#include <stdexcept>
#include <utility>

namespace rpf {
namespace {

void fail(const std::string& m) { throw std::runtime_error(m); }

int find_pos(const std::vector<int32_t>& ptr, const std::vector<int32_t>& col, int row, int c) {
  auto b = col.begin() + ptr[row], e = col.begin() + ptr[row + 1];
  auto it = std::lower_bound(b, e, c);
  if (it == e || *it != c) return -1;
  return (int)(it - col.begin());
}

// Minimum degree on the bus graph without the REF bus.  The degree of a bus
// is the number of state variables adjacent to it in the elimination graph
// (1 for PV, 2 for PQ neighbours).  Ties go to the lowest bus id.
std::vector<int> bus_min_degree(int nb, int ref, const std::vector<std::vector<int>>& adj0,
                                 const std::vector<int>& weight) {
  std::vector<std::set<int>> adj(nb);
  for (int i = 0; i < nb; ++i) {
    if (i == ref) continue;
    for (int j : adj0[i])
      if (j != ref && j != i) adj[i].insert(j);
  }
  std::vector<int> deg(nb, 0);
  std::set<std::pair<int, int>> pq;
  for (int i = 0; i < nb; ++i) {
    if (i == ref) continue;
    int d = 0;
    for (int j : adj[i]) d += weight[j];
    deg[i] = d;
    pq.insert({d, i});
  }
  std::vector<char> gone(nb, 0);
  std::vector<int> order;
  order.reserve(nb);
  while (!pq.empty()) {
    auto [d, v] = *pq.begin();
    pq.erase(pq.begin());
    gone[v] = 1;
    order.push_back(v);
    std::vector<int> nbrs(adj[v].begin(), adj[v].end());
    for (int a : nbrs) adj[a].erase(v);
    for (size_t x = 0; x < nbrs.size(); ++x)
      for (size_t y = x + 1; y < nbrs.size(); ++y) {
        adj[nbrs[x]].insert(nbrs[y]);
        adj[nbrs[y]].insert(nbrs[x]);
      }
    for (int a : nbrs) {
      int nd = 0;
      for (int j : adj[a]) nd += weight[j];
      if (nd != deg[a]) {
        pq.erase({deg[a], a});
        deg[a] = nd;
        pq.insert({nd, a});
      }
    }
    adj[v].clear();
  }
  return order;
}

Levels make_levels(const std::vector<int>& level) {
  Levels L;
  int nlev = 0;
  for (int v : level) nlev = std::max(nlev, v + 1);
  std::vector<int32_t> cnt(nlev + 1, 0);
  for (int v : level) cnt[v + 1]++;
  for (int k = 0; k < nlev; ++k) cnt[k + 1] += cnt[k];
  L.ptr = cnt;
  L.rows.assign(level.size(), 0);
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (size_t i = 0; i < level.size(); ++i) L.rows[fill[level[i]]++] = (int32_t)i;
  return L;
}

// CSR from per-row sorted lists
void to_csr(const std::vector<std::vector<int>>& rows, std::vector<int32_t>& ptr,
            std::vector<int32_t>& col) {
  ptr.assign(rows.size() + 1, 0);
  for (size_t i = 0; i < rows.size(); ++i) ptr[i + 1] = ptr[i] + (int32_t)rows[i].size();
  col.clear();
  col.reserve(ptr.back());
  for (auto& r : rows) col.insert(col.end(), r.begin(), r.end());
}

// gather lists from (slot, source) pairs; sources kept in insertion order
void to_lists(int nslots, std::vector<std::pair<int, int>>& pairs, std::vector<int32_t>& ptr,
              std::vector<int32_t>& src) {
  std::stable_sort(pairs.begin(), pairs.end(),
                   [](const auto& a, const auto& b) { return a.first < b.first; });
  ptr.assign(nslots + 1, 0);
  for (auto& p : pairs) ptr[p.first + 1]++;
  for (int i = 0; i < nslots; ++i) ptr[i + 1] += ptr[i];
  src.resize(pairs.size());
  for (size_t i = 0; i < pairs.size(); ++i) src[i] = pairs[i].second;
}

}  // namespace

Presolve build_presolve(const GridData& g, int subtree_max, int tail_max) {
  Presolve P;
  P.subtree_max = subtree_max;
  if (tail_max < 0 || tail_max > TAIL_MAX) fail("tail_max must be in [0, 128]");
  P.tail_max = tail_max;
  const int nb = g.nb, nl = g.nl, ng = g.ng;
  if (nb < 2 || nl < 1 || ng < 1) fail("grid needs nb >= 2, nl >= 1, ng >= 1");
  if ((int)g.bus_type.size() != nb || (int)g.br_from.size() != nl || (int)g.br_to.size() != nl ||
      (int)g.br_r.size() != nl || (int)g.br_x.size() != nl || (int)g.br_b.size() != nl ||
      (int)g.gen_bus.size() != ng || (int)g.c2.size() != ng || (int)g.c1.size() != ng ||
      (int)g.c0.size() != ng)
    fail("grid array sizes do not match nb/nl/ng");
  P.nb = nb; P.nl = nl; P.ng = ng; P.base_mva = g.base_mva;
  P.gen_at.assign(nb, -1);
  for (int k = 0; k < ng; ++k) {
    int b = g.gen_bus[k];
    if (b < 0 || b >= nb) fail("generator bus out of range");
    if (P.gen_at[b] >= 0) fail("more than one generator at a bus");
    P.gen_at[b] = k;
  }
  for (int i = 0; i < nb; ++i) {
    int t = g.bus_type[i];
    if (t == BUS_REF) {
      if (P.ref >= 0) fail("more than one REF bus");
      P.ref = i;
    } else if (t == BUS_PV) {
      P.pv.push_back(i);
    } else if (t == BUS_PQ) {
      P.pq.push_back(i);
    } else {
      fail("bus type must be 0 (PQ), 1 (PV) or 2 (REF)");
    }
    if ((t == BUS_REF || t == BUS_PV) && P.gen_at[i] < 0) fail("PV/REF bus without generator");
    if (t == BUS_PQ && P.gen_at[i] >= 0) fail("generator at a PQ bus");
  }
  if (P.ref < 0) fail("no REF bus");
  P.npv = (int)P.pv.size();
  P.npq = (int)P.pq.size();
  P.nx = P.npv + 2 * P.npq;
  P.nu = 1 + 2 * P.npv;
  P.m = 2 * nl + P.npq + P.npv + 2;
  P.nvar = P.nx + P.nu;
  const int nx = P.nx;
  if (nx < 1) fail("no state variables");

  std::vector<std::vector<int>> adj(nb);
  for (int l = 0; l < nl; ++l) {
    int f = g.br_from[l], t = g.br_to[l];
    if (f < 0 || f >= nb || t < 0 || t >= nb || f == t) fail("branch endpoints invalid");
    if (!(g.br_x[l] != 0.0 || g.br_r[l] != 0.0)) fail("branch with zero impedance");
    adj[f].push_back(t);
    adj[t].push_back(f);
  }
  for (auto& a : adj) {
    std::sort(a.begin(), a.end());
    if (std::adjacent_find(a.begin(), a.end()) != a.end()) fail("parallel branches are not supported");
  }

  // ------------------------------------------------------------ ordering
  std::vector<int> weight(nb, 0);
  for (int i = 0; i < nb; ++i) weight[i] = g.bus_type[i] == BUS_PQ ? 2 : (g.bus_type[i] == BUS_PV ? 1 : 0);
  std::vector<int> order = bus_min_degree(nb, P.ref, adj, weight);
  // state variables in elimination order: theta_i, then v_i for PQ buses
  std::vector<std::pair<int, int>> vars;   // (bus, is_v)
  for (int bus : order) {
    vars.push_back({bus, 0});
    if (g.bus_type[bus] == BUS_PQ) vars.push_back({bus, 1});
  }
  if ((int)vars.size() != nx) fail("internal: state count mismatch");
  std::vector<int> pv_pos(nb, -1), pq_pos(nb, -1);
  for (int k = 0; k < P.npv; ++k) pv_pos[P.pv[k]] = k;
  for (int k = 0; k < P.npq; ++k) pq_pos[P.pq[k]] = k;

  std::vector<int> parent;
  std::vector<std::vector<int>> lrow, urow;
  // number the variables in the order `vars` and compute the symbolic
  // factorization (elimination tree, row patterns of L and U)
  auto symbolic = [&]() {
    P.th_var.assign(nb, -1);
    P.v_var.assign(nb, -1);
    P.p_var.assign(nb, -1);
    P.rowP.assign(nb, -1);
    P.rowQ.assign(nb, -1);
    P.x_int2paper.assign(nx, -1);
    P.var_bus.assign(nx, -1);
    P.var_isv.assign(nx, 0);
    for (int c = 0; c < nx; ++c) {
      int bus = vars[c].first;
      P.var_bus[c] = bus;
      if (vars[c].second == 0) {
        P.th_var[bus] = c;
        P.rowP[bus] = c;
        P.x_int2paper[c] = g.bus_type[bus] == BUS_PV ? pv_pos[bus] : P.npv + pq_pos[bus];
      } else {
        P.v_var[bus] = c;
        P.rowQ[bus] = c;
        P.var_isv[c] = 1;
        P.x_int2paper[c] = P.npv + P.npq + pq_pos[bus];
      }
    }
    P.v_var[P.ref] = nx;
    for (int k = 0; k < P.npv; ++k) {
      P.v_var[P.pv[k]] = nx + 1 + k;
      P.p_var[P.pv[k]] = nx + 1 + P.npv + k;
    }
    std::vector<std::vector<int>> arow(nx);
    for (int r = 0; r < nx; ++r) {
      int i = P.var_bus[r];
      auto add_bus = [&](int bb) {
        if (P.th_var[bb] >= 0) arow[r].push_back(P.th_var[bb]);
        if (g.bus_type[bb] == BUS_PQ) arow[r].push_back(P.v_var[bb]);
      };
      add_bus(i);
      for (int j : adj[i]) add_bus(j);
      std::sort(arow[r].begin(), arow[r].end());
    }
    parent.assign(nx, -1);
    std::vector<int> ancestor(nx, -1);
    for (int i = 0; i < nx; ++i)
      for (int k : arow[i]) {
        if (k >= i) break;
        int r = k;
        while (ancestor[r] != -1 && ancestor[r] != i) {
          int nxt = ancestor[r];
          ancestor[r] = i;
          r = nxt;
        }
        if (ancestor[r] == -1) {
          ancestor[r] = i;
          parent[r] = i;
        }
      }
    lrow.assign(nx, {});
    urow.assign(nx, {});
    std::vector<int> mark(nx, -1);
    for (int i = 0; i < nx; ++i) {
      mark[i] = i;
      for (int k : arow[i]) {
        if (k >= i) break;
        int j = k;
        while (mark[j] != i) {
          lrow[i].push_back(j);
          mark[j] = i;
          j = parent[j];
          if (j < 0) fail("internal: broken elimination tree");
        }
      }
      std::sort(lrow[i].begin(), lrow[i].end());
    }
    for (int i = 0; i < nx; ++i)
      for (int k : lrow[i]) urow[k].push_back(i);   // ascending i -> sorted
  };
  symbolic();

  // ------------------------------------------------ subtree partition
  // Subtrees of the elimination tree with at most subtree_max rows are
  // independent in the forward solves and in the refactorization; they are
  // packed into contiguous row ranges (packs), and the remaining "top" rows
  // (ancestors of the packs) are numbered last.  Any topological order of
  // the elimination tree has the same fill, so the factor pattern is only
  // permuted.
  {
    const int smax = std::max(1, P.subtree_max);
    std::vector<int> size(nx, 1);
    for (int i = 0; i < nx; ++i)
      if (parent[i] >= 0) size[parent[i]] += size[i];
    std::vector<int> root_of(nx, -1);
    std::vector<char> is_top(nx, 0);
    for (int i = nx - 1; i >= 0; --i) {
      if (size[i] > smax) {
        is_top[i] = 1;
      } else if (parent[i] < 0 || size[parent[i]] > smax) {
        root_of[i] = i;
      } else {
        root_of[i] = root_of[parent[i]];
      }
    }
    // packs: consecutive subtree roots (ascending) up to smax rows each
    std::vector<int> pack_of_root(nx, -1);
    int npk = 0, fillc = 0;
    for (int i = 0; i < nx; ++i)
      if (root_of[i] == i) {
        if (npk == 0 || fillc + size[i] > smax) {
          ++npk;
          fillc = 0;
        }
        pack_of_root[i] = npk - 1;
        fillc += size[i];
      }
    std::vector<int> key(nx);
    for (int i = 0; i < nx; ++i) key[i] = is_top[i] ? npk : pack_of_root[root_of[i]];
    std::vector<int> newo(nx);
    std::iota(newo.begin(), newo.end(), 0);
    std::stable_sort(newo.begin(), newo.end(), [&](int x0, int x1) { return key[x0] < key[x1]; });
    std::vector<std::pair<int, int>> v2(nx);
    for (int c = 0; c < nx; ++c) v2[c] = vars[newo[c]];
    vars = v2;
    P.pack_ptr.assign(npk + 1, 0);
    for (int i = 0; i < nx; ++i)
      if (!is_top[i]) P.pack_ptr[pack_of_root[root_of[i]] + 1]++;
    for (int q = 0; q < npk; ++q) P.pack_ptr[q + 1] += P.pack_ptr[q];
    P.t0 = P.pack_ptr[npk];
  }
  symbolic();
  std::vector<std::vector<int>> lurow(nx);
  P.lu_diag.assign(nx, 0);
  for (int i = 0; i < nx; ++i) {
    lurow[i] = lrow[i];
    lurow[i].push_back(i);
    lurow[i].insert(lurow[i].end(), urow[i].begin(), urow[i].end());
    P.max_lu_row = std::max(P.max_lu_row, (int)lurow[i].size());
  }
  to_csr(lurow, P.lu_ptr, P.lu_col);
  for (int i = 0; i < nx; ++i) P.lu_diag[i] = P.lu_ptr[i] + (int)lrow[i].size();
  // transposed factor has the same (symmetric) pattern; sources swap (i,c)
  P.lut_ptr = P.lu_ptr;
  P.lut_col = P.lu_col;
  P.lut_diag = P.lu_diag;
  P.lut_src.assign(P.lu_col.size(), -1);
  for (int i = 0; i < nx; ++i)
    for (int p = P.lu_ptr[i]; p < P.lu_ptr[i + 1]; ++p) {
      int c = P.lu_col[p];
      int q = find_pos(P.lu_ptr, P.lu_col, c, i);
      if (q < 0) fail("internal: pattern not symmetric");
      P.lut_src[p] = q;
    }

  // --------------------------------------------------------------- levels
  std::vector<int> lev(nx, 0), ulev(nx, 0);
  for (int i = 0; i < nx; ++i) {
    int v = 0;
    for (int k : lrow[i]) v = std::max(v, lev[k] + 1);
    lev[i] = v;
  }
  for (int i = nx - 1; i >= 0; --i) {
    int v = 0;
    for (int j : urow[i]) v = std::max(v, ulev[j] + 1);
    ulev[i] = v;
  }
  P.lev_lo = make_levels(lev);
  P.lev_up = make_levels(ulev);

  // ------------------------------------------- partition level lists
  {
    const int t0 = P.t0;
    const int npk = (int)P.pack_ptr.size() - 1;
    P.lo_split.assign(nx, 0);
    P.up_split.assign(nx, 0);
    for (int i = 0; i < nx; ++i) {
      int p = P.lu_ptr[i];
      while (p < P.lu_diag[i] && P.lu_col[p] < t0) ++p;
      P.lo_split[i] = p;
      int q = P.lu_diag[i] + 1;
      while (q < P.lu_ptr[i + 1] && P.lu_col[q] < t0) ++q;
      P.up_split[i] = q;
    }
    // every LDS index of the partitioned solves stays inside its block:
    // pack rows reference their own pack or the top part, top rows
    // reference packs (below t0) only through their first lower entries
    for (int q = 0; q + 1 < (int)P.pack_ptr.size(); ++q)
      for (int i = P.pack_ptr[q]; i < P.pack_ptr[q + 1]; ++i)
        for (int p = P.lu_ptr[i]; p < P.lu_ptr[i + 1]; ++p) {
          int c = P.lu_col[p];
          bool own = c >= P.pack_ptr[q] && c < P.pack_ptr[q + 1];
          if (!own && c < t0) fail("internal: pack row references another pack");
          if (c >= t0 && p < P.lu_diag[i]) fail("internal: pack row has a top column below its diagonal");
        }
    for (int i = t0; i < nx; ++i)
      for (int p = P.lu_diag[i]; p < P.lu_ptr[i + 1]; ++p)
        if (P.lu_col[p] < t0) fail("internal: top row references a pack above its diagonal");
    // forward / backward levels inside each pack (pack-local dependencies)
    P.pk_flev.assign(1, 0);
    P.pk_blev.assign(1, 0);
    P.pk_flev_off.assign(npk + 1, 0);
    P.pk_blev_off.assign(npk + 1, 0);
    P.pk_frows.clear();
    P.pk_brows.clear();
    std::vector<int> lv(nx, 0);
    for (int q = 0; q < npk; ++q) {
      const int r0 = P.pack_ptr[q], r1 = P.pack_ptr[q + 1];
      int nlv = 0;
      for (int i = r0; i < r1; ++i) {
        int v = 0;
        for (int k : lrow[i]) {
          if (k < r0 || k >= r1) fail("internal: pack dependency leaves the pack");
          v = std::max(v, lv[k] + 1);
        }
        lv[i] = v;
        nlv = std::max(nlv, v + 1);
      }
      std::vector<std::vector<int>> byl(nlv);
      for (int i = r0; i < r1; ++i) byl[lv[i]].push_back(i);
      for (auto& b : byl) {
        P.pk_frows.insert(P.pk_frows.end(), b.begin(), b.end());
        P.pk_flev.push_back((int)P.pk_frows.size());
      }
      P.pk_flev_off[q + 1] = (int)P.pk_flev.size() - 1;
      int nbl = 0;
      for (int i = r1 - 1; i >= r0; --i) {
        int v = 0;
        for (int j : urow[i])
          if (j < r1) v = std::max(v, lv[j] + 1);
        lv[i] = v;
        nbl = std::max(nbl, v + 1);
      }
      std::vector<std::vector<int>> byb(nbl);
      for (int i = r0; i < r1; ++i) byb[lv[i]].push_back(i);
      for (auto& b : byb) {
        P.pk_brows.insert(P.pk_brows.end(), b.begin(), b.end());
        P.pk_blev.push_back((int)P.pk_brows.size());
      }
      P.pk_blev_off[q + 1] = (int)P.pk_blev.size() - 1;
    }
    // staged programs (pack-local columns fit int16: packs hold at most
    // subtree_max <= 32767 rows)
    if (P.subtree_max > 32767) fail("subtree_max must stay below 32768");
    P.pkf_rp.assign(t0 + 1, 0);
    P.pkb_rp.assign(t0 + 1, 0);
    P.pkf_pos.clear(); P.pkf_col.clear(); P.pkb_pos.clear(); P.pkb_col.clear();
    for (int q = 0; q < npk; ++q) {
      const int r0 = P.pack_ptr[q], r1 = P.pack_ptr[q + 1];
      for (int i = r0; i < r1; ++i) {
        for (int p = P.lu_ptr[i]; p < P.lu_diag[i]; ++p) {
          P.pkf_pos.push_back(p);
          P.pkf_col.push_back((int16_t)(P.lu_col[p] - r0));
        }
        P.pkf_rp[i + 1] = (int32_t)P.pkf_pos.size();
        for (int p = P.lu_diag[i] + 1; p < P.up_split[i]; ++p) {
          P.pkb_pos.push_back(p);
          P.pkb_col.push_back((int16_t)(P.lu_col[p] - r0));
        }
        P.pkb_rp[i + 1] = (int32_t)P.pkb_pos.size();
      }
    }
    // dense tails and the batched programs (see Presolve::ptl_*)
    {
      const int TD = P.tail_max;
      P.ptl_off.assign(npk + 1, 0);
      P.ptl_eoff.assign(npk + 1, 0);
      P.ptl_rows.clear(); P.ptl_pos.clear(); P.ptl_dense.clear();
      P.ptf_lev.assign(1, 0); P.ptb_lev.assign(1, 0);
      P.ptf_lev_off.assign(npk + 1, 0); P.ptb_lev_off.assign(npk + 1, 0);
      P.ptf_rows.clear(); P.ptb_rows.clear();
      P.ptf_rp.assign(t0 + 1, 0); P.ptb_rp.assign(t0 + 1, 0);
      P.ptf_pos.clear(); P.ptf_col.clear(); P.ptb_pos.clear(); P.ptb_col.clear();
      P.rft_ptr.assign(1, 0);
      P.rft_pos.clear();
      std::vector<int> hgt(nx, 0), tix(nx, -1), blv(nx, 0);
      for (int q = 0; q < npk; ++q) {
        const int r0 = P.pack_ptr[q], r1 = P.pack_ptr[q + 1];
        int hmax = 0;
        for (int i = r0; i < r1; ++i) {
          int v = 0;
          for (int k : lrow[i]) v = std::max(v, hgt[k] + 1);
          hgt[i] = v;
          hmax = std::max(hmax, v);
        }
        // cut hc: the fewest levels left with at most TD rows at heights >= hc
        std::vector<int> cnt(hmax + 1, 0);
        for (int i = r0; i < r1; ++i) cnt[hgt[i]]++;
        int hc = hmax + 1, acc = 0;
        while (hc > 0 && acc + cnt[hc - 1] <= TD) acc += cnt[--hc];
        int nT = 0;
        for (int i = r0; i < r1; ++i) {
          tix[i] = hgt[i] >= hc ? nT++ : -1;
          if (tix[i] >= 0) P.ptl_rows.push_back((int16_t)(i - r0));
        }
        P.ptl_off[q + 1] = (int)P.ptl_rows.size();
        // an ancestor-closed T: the parent of a T row is in T (heights grow
        // towards the root), so no other row depends on a T row going up
        for (int i = r0; i < r1; ++i)
          if (tix[i] < 0)
            for (int k : lrow[i])
              if (tix[k] >= 0) fail("internal: tail rows are not ancestor-closed");
        for (int i = r0; i < r1; ++i) {
          if (tix[i] < 0) continue;
          for (int p = P.lu_ptr[i]; p < P.lu_ptr[i + 1]; ++p) {
            const int c = P.lu_col[p];
            if (c >= r0 && c < r1 && tix[c] >= 0) {
              P.ptl_pos.push_back(p);
              P.ptl_dense.push_back(tix[i] * TAIL_MAX + tix[c]);
            }
          }
        }
        P.ptl_eoff[q + 1] = (int)P.ptl_pos.size();
        // right-looking lists of the tail block for the refactorization
        {
          std::vector<int> trow;
          for (int i = r0; i < r1; ++i)
            if (tix[i] >= 0) trow.push_back(i);
          for (int b = 0; b < nT; ++b) {
            const int k = trow[b];
            for (int b2 = b + 1; b2 < nT; ++b2) {
              const int pos = find_pos(P.lu_ptr, P.lu_col, trow[b2], k);
              if (pos >= 0) P.rft_pos.push_back(pos);
            }
            P.rft_ptr.push_back((int)P.rft_pos.size());
          }
        }
        // forward: other rows by height, then the T rows as one level
        std::vector<std::vector<int>> byl(hc + (nT > 0 ? 1 : 0));
        for (int i = r0; i < r1; ++i) byl[tix[i] >= 0 ? hc : hgt[i]].push_back(i);
        for (auto& b : byl) {
          if (b.empty()) continue;
          P.ptf_rows.insert(P.ptf_rows.end(), b.begin(), b.end());
          P.ptf_lev.push_back((int)P.ptf_rows.size());
        }
        P.ptf_lev_off[q + 1] = (int)P.ptf_lev.size() - 1;
        // backward: the other rows, levels over their dependencies among
        // themselves (the T rows are done first)
        int nbl = 0;
        for (int i = r1 - 1; i >= r0; --i) {
          if (tix[i] >= 0) continue;
          int v = 0;
          for (int j : urow[i])
            if (j < r1 && tix[j] < 0) v = std::max(v, blv[j] + 1);
          blv[i] = v;
          nbl = std::max(nbl, v + 1);
        }
        std::vector<std::vector<int>> byb(nbl);
        for (int i = r0; i < r1; ++i)
          if (tix[i] < 0) byb[blv[i]].push_back(i);
        for (auto& b : byb) {
          P.ptb_rows.insert(P.ptb_rows.end(), b.begin(), b.end());
          P.ptb_lev.push_back((int)P.ptb_rows.size());
        }
        P.ptb_lev_off[q + 1] = (int)P.ptb_lev.size() - 1;
        // staged entries: forward, a T row keeps only its columns outside T;
        // backward, T rows have none
        for (int i = r0; i < r1; ++i) {
          for (int p = P.lu_ptr[i]; p < P.lu_diag[i]; ++p) {
            const int c = P.lu_col[p];
            if (tix[i] >= 0 && tix[c] >= 0) continue;
            P.ptf_pos.push_back(p);
            P.ptf_col.push_back((int16_t)(c - r0));
          }
          P.ptf_rp[i + 1] = (int32_t)P.ptf_pos.size();
          if (tix[i] < 0) {
            for (int p = P.lu_diag[i] + 1; p < P.up_split[i]; ++p) {
              P.ptb_pos.push_back(p);
              P.ptb_col.push_back((int16_t)(P.lu_col[p] - r0));
            }
          }
          P.ptb_rp[i + 1] = (int32_t)P.ptb_pos.size();
        }
      }
    }
    // top part: forward levels over top-internal lower entries, backward over upper
    std::vector<int> tl(nx, 0);
    int ntf = 0, ntb = 0;
    for (int i = t0; i < nx; ++i) {
      int v = 0;
      for (int k : lrow[i])
        if (k >= t0) v = std::max(v, tl[k] + 1);
      tl[i] = v;
      ntf = std::max(ntf, v + 1);
    }
    std::vector<std::vector<int>> tf(ntf);
    for (int i = t0; i < nx; ++i) tf[tl[i]].push_back(i);
    for (int i = nx - 1; i >= t0; --i) {
      int v = 0;
      for (int j : urow[i]) v = std::max(v, tl[j] + 1);
      tl[i] = v;
      ntb = std::max(ntb, v + 1);
    }
    std::vector<std::vector<int>> tb(ntb);
    for (int i = t0; i < nx; ++i) tb[tl[i]].push_back(i);
    P.top_flev.assign(1, 0);
    P.top_frows.clear();
    for (auto& b : tf) {
      P.top_frows.insert(P.top_frows.end(), b.begin(), b.end());
      P.top_flev.push_back((int)P.top_frows.size());
    }
    P.top_blev.assign(1, 0);
    P.top_brows.clear();
    for (auto& b : tb) {
      P.top_brows.insert(P.top_brows.end(), b.begin(), b.end());
      P.top_blev.push_back((int)P.top_brows.size());
    }
    // dense top block positions: for each top row, LU positions with col >= t0
    const int s = nx - t0;
    P.ntop = s;
    P.top_pos.clear();
    P.top_dense.clear();
    for (int i = t0; i < nx; ++i)
      for (int p = P.lo_split[i]; p < P.lu_ptr[i + 1]; ++p) {
        P.top_pos.push_back(p);
        P.top_dense.push_back((int64_t)(i - t0) * s + (P.lu_col[p] - t0));
      }
  }

  // -------------------------------------------------- refactorization map
  const int64_t nnz = (int64_t)P.lu_col.size();
  P.upd_ptr.assign(nnz + 1, 0);
  std::vector<int32_t> tg;
  for (int i = 0; i < nx; ++i) {
    for (int p = P.lu_ptr[i]; p < P.lu_ptr[i + 1]; ++p) {
      if (p < P.lu_diag[i]) {
        int k = P.lu_col[p];
        for (int q = P.lu_diag[k] + 1; q < P.lu_ptr[k + 1]; ++q) {
          int t = find_pos(P.lu_ptr, P.lu_col, i, P.lu_col[q]);
          if (t < 0) fail("internal: symbolic fill incomplete");
          tg.push_back(t);
        }
      }
      P.upd_ptr[p + 1] = (int64_t)tg.size();
    }
  }
  P.upd_tgt = std::move(tg);
  // U-row start of the pivot row of every L entry (lu_diag[col] + 1)
  P.rf_ustart.assign(nnz, 0);
  for (int i = 0; i < nx; ++i)
    for (int p = P.lu_ptr[i]; p < P.lu_diag[i]; ++p) P.rf_ustart[p] = P.lu_diag[P.lu_col[p]] + 1;

  // ------------------------------------------------------- branch locals
  P.br_var.assign((size_t)nl * 4, -1);
  for (int l = 0; l < nl; ++l) {
    int f = g.br_from[l], t = g.br_to[l];
    P.br_var[4 * l + 0] = P.th_var[f];
    P.br_var[4 * l + 1] = P.th_var[t];
    P.br_var[4 * l + 2] = P.v_var[f];
    P.br_var[4 * l + 3] = P.v_var[t];
  }
  {
    std::vector<std::vector<int>> inc(nb);
    for (int l = 0; l < nl; ++l) {
      inc[g.br_from[l]].push_back(2 * l);
      inc[g.br_to[l]].push_back(2 * l + 1);
    }
    to_csr(inc, P.inc_ptr, P.inc_end);
  }
  auto end_bus = [&](int l, int e) { return e == 0 ? g.br_from[l] : g.br_to[l]; };

  // ------------------------------------ J_x, J_u gather lists and pattern
  {
    std::vector<std::pair<int, int>> jx_pairs;
    std::map<std::pair<int, int>, std::vector<int>> ju_map;   // (row, ucol) -> sources
    for (int l = 0; l < nl; ++l)
      for (int e = 0; e < 2; ++e) {
        int i = end_bus(l, e);
        for (int E = 0; E < 2; ++E) {
          int row = E == 0 ? P.rowP[i] : P.rowQ[i];
          if (row < 0) continue;
          int eq = 2 * e + E;
          for (int k = 0; k < 4; ++k) {
            int c = P.br_var[4 * l + k];
            if (c < 0) continue;
            int src = l * RECW + 4 + 4 * eq + k;
            if (c < nx) {
              int pos = find_pos(P.lu_ptr, P.lu_col, row, c);
              if (pos < 0) fail("internal: J_x entry outside pattern");
              jx_pairs.push_back({pos, src});
            } else {
              ju_map[{row, c - nx}].push_back(src);
            }
          }
        }
      }
    for (int k = 0; k < P.npv; ++k) {
      int i = P.pv[k];
      ju_map[{P.rowP[i], 1 + P.npv + k}];   // constant -1 entry
    }
    to_lists((int)nnz, jx_pairs, P.jx_src_ptr, P.jx_src);
    P.ju_ptr.assign(nx + 1, 0);
    for (auto& kv : ju_map) P.ju_ptr[kv.first.first + 1]++;
    for (int r = 0; r < nx; ++r) P.ju_ptr[r + 1] += P.ju_ptr[r];
    P.ju_src_ptr.assign(1, 0);
    for (auto& kv : ju_map) {
      P.ju_col.push_back(kv.first.second);
      for (int s : kv.second) P.ju_src.push_back(s);
      P.ju_src_ptr.push_back((int32_t)P.ju_src.size());
      bool isp = kv.first.second > P.npv;   // p_pv column
      P.ju_const.push_back(isp ? -1.0 : 0.0);
    }
    // transpose of J_u: CSR over controls
    const int nju = (int)P.ju_col.size();
    P.jut_ptr.assign(P.nu + 1, 0);
    for (int p = 0; p < nju; ++p) P.jut_ptr[P.ju_col[p] + 1]++;
    for (int c = 0; c < P.nu; ++c) P.jut_ptr[c + 1] += P.jut_ptr[c];
    P.jut_col.assign(nju, 0);
    P.jut_srcpos.assign(nju, 0);
    std::vector<int32_t> fill(P.jut_ptr.begin(), P.jut_ptr.end() - 1);
    for (int r = 0; r < nx; ++r)
      for (int p = P.ju_ptr[r]; p < P.ju_ptr[r + 1]; ++p) {
        int c = P.ju_col[p];
        P.jut_col[fill[c]] = r;
        P.jut_srcpos[fill[c]] = p;
        fill[c]++;
      }
  }

  // -------------------------------------------------------------- g rows
  {
    P.row_bus.assign(nx, -1);
    P.row_isq.assign(nx, 0);
    P.row_pvar.assign(nx, -1);
    std::vector<std::pair<int, int>> pairs;
    for (int i = 0; i < nb; ++i)
      for (int E = 0; E < 2; ++E) {
        int row = E == 0 ? P.rowP[i] : P.rowQ[i];
        if (row < 0) continue;
        P.row_bus[row] = i;
        P.row_isq[row] = E;
        if (E == 0 && g.bus_type[i] == BUS_PV) P.row_pvar[row] = P.p_var[i] - nx;
        for (int q = P.inc_ptr[i]; q < P.inc_ptr[i + 1]; ++q) {
          int l = P.inc_end[q] >> 1, e = P.inc_end[q] & 1;
          pairs.push_back({row, l * RECW + 2 * e + E});
        }
      }
    to_lists(nx, pairs, P.g_src_ptr, P.g_src);
  }

  // ------------------------------------------- rank-one constraint rows G
  {
    P.nr1 = 2 + P.npv;
    P.r1_bus.push_back(P.ref);
    P.r1_isq.push_back(0);
    P.r1_bus.push_back(P.ref);
    P.r1_isq.push_back(1);
    for (int k = 0; k < P.npv; ++k) {
      P.r1_bus.push_back(P.pv[k]);
      P.r1_isq.push_back(1);
    }
    std::map<std::pair<int, int>, std::vector<int>> gm;
    for (int r = 0; r < P.nr1; ++r) {
      int i = P.r1_bus[r], E = P.r1_isq[r];
      for (int q = P.inc_ptr[i]; q < P.inc_ptr[i + 1]; ++q) {
        int l = P.inc_end[q] >> 1, e = P.inc_end[q] & 1;
        for (int k = 0; k < 4; ++k) {
          int c = P.br_var[4 * l + k];
          if (c < 0) continue;
          gm[{r, c}].push_back(l * RECW + 4 + 4 * (2 * e + E) + k);
        }
      }
    }
    P.G_ptr.assign(P.nr1 + 1, 0);
    P.G_src_ptr.assign(1, 0);
    for (auto& kv : gm) {
      P.G_ptr[kv.first.first + 1]++;
      P.G_col.push_back(kv.first.second);
      for (int s : kv.second) P.G_src.push_back(s);
      P.G_src_ptr.push_back((int32_t)P.G_src.size());
    }
    for (int r = 0; r < P.nr1; ++r) P.G_ptr[r + 1] += P.G_ptr[r];
    const int ngz = (int)P.G_col.size();
    P.Gt_ptr.assign(P.nvar + 1, 0);
    for (int p = 0; p < ngz; ++p) P.Gt_ptr[P.G_col[p] + 1]++;
    for (int c = 0; c < P.nvar; ++c) P.Gt_ptr[c + 1] += P.Gt_ptr[c];
    P.Gt_col.assign(ngz, 0);
    P.Gt_srcpos.assign(ngz, 0);
    std::vector<int32_t> fill(P.Gt_ptr.begin(), P.Gt_ptr.end() - 1);
    for (int r = 0; r < P.nr1; ++r)
      for (int p = P.G_ptr[r]; p < P.G_ptr[r + 1]; ++p) {
        int c = P.G_col[p];
        P.Gt_col[fill[c]] = r;
        P.Gt_srcpos[fill[c]] = p;
        fill[c]++;
      }
  }

  // ------------------------------------------------- Lagrangian Hessian K
  {
    std::map<std::pair<int, int>, std::vector<int>> km;
    for (int c = 0; c < P.nvar; ++c) km[{c, c}];
    for (int l = 0; l < nl; ++l)
      for (int k1 = 0; k1 < 4; ++k1) {
        int c1 = P.br_var[4 * l + k1];
        if (c1 < 0) continue;
        for (int k2 = 0; k2 < 4; ++k2) {
          int c2 = P.br_var[4 * l + k2];
          if (c2 < 0) continue;
          km[{c1, c2}].push_back(l * WREC + 4 * k1 + k2);
        }
      }
    P.K_ptr.assign(P.nvar + 1, 0);
    P.K_src_ptr.assign(1, 0);
    P.K_diag.assign(P.nvar, -1);
    for (auto& kv : km) {
      int r = kv.first.first, c = kv.first.second;
      P.K_ptr[r + 1]++;
      if (r == c) P.K_diag[r] = (int)P.K_col.size();
      P.K_col.push_back(c);
      for (int s : kv.second) P.K_src.push_back(s);
      P.K_src_ptr.push_back((int32_t)P.K_src.size());
    }
    for (int r = 0; r < P.nvar; ++r) P.K_ptr[r + 1] += P.K_ptr[r];
    std::vector<std::pair<int, int>> vg;
    for (int l = 0; l < nl; ++l)
      for (int k = 0; k < 4; ++k) {
        int c = P.br_var[4 * l + k];
        if (c >= 0) vg.push_back({c, l * WREC + 16 + k});
      }
    to_lists(P.nvar, vg, P.vg_src_ptr, P.vg_src);
  }
  return P;
}

PresolveStats stats(const Presolve& p) {
  PresolveStats s{};
  int64_t nj = 0;
  for (size_t i = 0; i + 1 < p.jx_src_ptr.size(); ++i) nj += p.jx_src_ptr[i + 1] > p.jx_src_ptr[i];
  s.nnz_jx = nj;
  s.nnz_lu = (int64_t)p.lu_col.size();
  s.nlev_lo = p.lev_lo.nlev();
  s.nlev_up = p.lev_up.nlev();
  s.max_lu_row = p.max_lu_row;
  s.refactor_updates = (int64_t)p.upd_tgt.size();
  s.nnz_ju = (int64_t)p.ju_col.size();
  s.nnz_k = (int64_t)p.K_col.size();
  s.nnz_g = (int64_t)p.G_col.size();
  s.npacks = (int64_t)p.pack_ptr.size() - 1;
  s.ntop = p.ntop;
  int64_t mx = 0;
  for (int64_t q = 0; q < s.npacks; ++q)
    mx = std::max<int64_t>(mx, p.pk_flev_off[q + 1] - p.pk_flev_off[q]);
  s.max_pack_levels = mx;
  int64_t mf = 0, mb = 0;
  for (size_t q = 0; q + 1 < p.ptf_lev_off.size(); ++q) {
    mf = std::max<int64_t>(mf, p.ptf_lev_off[q + 1] - p.ptf_lev_off[q]);
    mb = std::max<int64_t>(mb, p.ptb_lev_off[q + 1] - p.ptb_lev_off[q]);
  }
  s.max_tail_fwd_levels = mf;
  s.max_tail_bwd_levels = mb;
  s.tail_rows = (int64_t)p.ptl_rows.size();
  s.top_levels = (int64_t)p.top_flev.size() - 1;
  return s;
}

}  // namespace rpf
