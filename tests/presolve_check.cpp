// Host check of the symbolic presolve (built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_presolve_sanitized.py): reads a
// grid file, builds the presolve and validates every solve schedule --
// each row of a level reads only rows finished in earlier levels (or, in a
// pack's backward program, rows of its dense tail, which are solved first)
// -- and that each pack program stages exactly the entries it must.
// Prints the presolve statistics as one line of integers.
//
// Grid file (little-endian): int32 nb, nl, ng; float64 base_mva; int32
// bus_type[nb], br_from[nl], br_to[nl], gen_bus[ng]; float64 br_r[nl],
// br_x[nl], br_b[nl], c2[ng], c1[ng], c0[ng].
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <stdexcept>
#include <string>
#include <vector>

#include "../paper_2110_02590_amd/csrc/presolve.hpp"

namespace {

template <class T>
void read_vec(std::ifstream& f, std::vector<T>& v, int n) {
  v.resize(n);
  if (n > 0) f.read(reinterpret_cast<char*>(v.data()), sizeof(T) * n);
  if (!f) throw std::runtime_error("grid file truncated");
}

void check(bool ok, const std::string& what) {
  if (!ok) throw std::runtime_error(what);
}

// a schedule over rows: level of each row (-1 when not scheduled), each row
// scheduled at most once
std::vector<int> levels_of(int n, const std::vector<int32_t>& ptr, const std::vector<int32_t>& rows,
                           const std::string& name) {
  std::vector<int> lv(n, -1);
  for (size_t k = 0; k + 1 < ptr.size(); ++k)
    for (int e = ptr[k]; e < ptr[k + 1]; ++e) {
      const int r = rows[e];
      check(r >= 0 && r < n, name + ": row out of range");
      check(lv[r] < 0, name + ": row scheduled twice");
      lv[r] = (int)k;
    }
  return lv;
}

void check_global(const rpf::Presolve& P) {
  const int nx = P.nx;
  const auto lo = levels_of(nx, P.lev_lo.ptr, P.lev_lo.rows, "forward schedule");
  const auto up = levels_of(nx, P.lev_up.ptr, P.lev_up.rows, "backward schedule");
  for (int i = 0; i < nx; ++i) {
    check(lo[i] >= 0 && up[i] >= 0, "a row is missing from a schedule");
    check(P.lu_col[P.lu_diag[i]] == i, "diagonal position");
    for (int p = P.lu_ptr[i]; p < P.lu_diag[i]; ++p)
      check(lo[P.lu_col[p]] < lo[i], "forward schedule reads an unfinished row");
    for (int p = P.lu_diag[i] + 1; p < P.lu_ptr[i + 1]; ++p)
      check(up[P.lu_col[p]] < up[i], "backward schedule reads an unfinished row");
  }
}

void check_packs(const rpf::Presolve& P) {
  const int npk = (int)P.pack_ptr.size() - 1;
  check(P.pack_ptr[npk] == P.t0, "packs end at the top part");
  std::vector<int> fl(P.nx, -1), bl(P.nx, -1), tail(P.nx, 0);
  for (int q = 0; q < npk; ++q) {
    const int r0 = P.pack_ptr[q], r1 = P.pack_ptr[q + 1];
    check(r1 - r0 <= P.subtree_max, "pack above the subtree limit");
    const int nT = P.ptl_off[q + 1] - P.ptl_off[q];
    check(nT <= P.tail_max && P.tail_max <= rpf::TAIL_MAX, "tail above its limit");
    for (int b = P.ptl_off[q]; b < P.ptl_off[q + 1]; ++b) {
      const int r = r0 + P.ptl_rows[b];
      check(r >= r0 && r < r1, "tail row outside its pack");
      tail[r] = 1;
    }
    for (int e = P.ptl_eoff[q]; e < P.ptl_eoff[q + 1]; ++e) {
      const int d = P.ptl_dense[e];
      check(d >= 0 && d / rpf::TAIL_MAX < nT && d % rpf::TAIL_MAX < nT, "tail entry outside the tail block");
    }
    // forward program: every pack row once
    for (int k = P.ptf_lev_off[q]; k < P.ptf_lev_off[q + 1]; ++k)
      for (int e = P.ptf_lev[k]; e < P.ptf_lev[k + 1]; ++e) {
        const int r = P.ptf_rows[e];
        check(r >= r0 && r < r1 && fl[r] < 0, "forward program row");
        fl[r] = k;
      }
    for (int k = P.ptb_lev_off[q]; k < P.ptb_lev_off[q + 1]; ++k)
      for (int e = P.ptb_lev[k]; e < P.ptb_lev[k + 1]; ++e) {
        const int r = P.ptb_rows[e];
        check(r >= r0 && r < r1 && bl[r] < 0 && !tail[r], "backward program row");
        bl[r] = k;
      }
    for (int i = r0; i < r1; ++i) {
      check(fl[i] >= 0, "pack row missing from its forward program");
      check(tail[i] || bl[i] >= 0, "pack row missing from its backward program");
      // forward: the staged entries are the row's L entries, less those
      // inside the tail block for a tail row; each reads an earlier level
      int want = 0;
      for (int p = P.lu_ptr[i]; p < P.lu_diag[i]; ++p) {
        const int c = P.lu_col[p];
        check(c >= r0 && c < i, "L entry of a pack row outside its pack");
        if (!(tail[i] && tail[c])) ++want;
      }
      check(P.ptf_rp[i + 1] - P.ptf_rp[i] == want, "forward program stages the wrong entries");
      for (int e = P.ptf_rp[i]; e < P.ptf_rp[i + 1]; ++e) {
        const int p = P.ptf_pos[e], c = r0 + P.ptf_col[e];
        check(p >= P.lu_ptr[i] && p < P.lu_diag[i] && P.lu_col[p] == c, "forward entry position");
        check(fl[c] < fl[i], "forward program reads an unfinished row");
      }
      // backward: a non-tail row's U entries inside the pack, each reading a
      // tail row or a row of an earlier level
      if (!tail[i]) {
        check(P.ptb_rp[i + 1] - P.ptb_rp[i] == P.up_split[i] - P.lu_diag[i] - 1,
              "backward program stages the wrong entries");
        for (int e = P.ptb_rp[i]; e < P.ptb_rp[i + 1]; ++e) {
          const int p = P.ptb_pos[e], c = r0 + P.ptb_col[e];
          check(p > P.lu_diag[i] && p < P.up_split[i] && P.lu_col[p] == c, "backward entry position");
          check(c < r1, "backward entry outside the pack");
          check(tail[c] || bl[c] < bl[i], "backward program reads an unfinished row");
        }
      } else {
        check(P.ptb_rp[i + 1] == P.ptb_rp[i], "a tail row has backward entries");
      }
    }
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s grid.bin\n", argv[0]);
    return 2;
  }
  try {
    std::ifstream f(argv[1], std::ios::binary);
    check((bool)f, "cannot open the grid file");
    rpf::GridData g;
    f.read(reinterpret_cast<char*>(&g.nb), 4);
    f.read(reinterpret_cast<char*>(&g.nl), 4);
    f.read(reinterpret_cast<char*>(&g.ng), 4);
    f.read(reinterpret_cast<char*>(&g.base_mva), 8);
    check((bool)f && g.nb > 0 && g.nl >= 0 && g.ng > 0, "grid header");
    read_vec(f, g.bus_type, g.nb);
    read_vec(f, g.br_from, g.nl);
    read_vec(f, g.br_to, g.nl);
    read_vec(f, g.gen_bus, g.ng);
    read_vec(f, g.br_r, g.nl);
    read_vec(f, g.br_x, g.nl);
    read_vec(f, g.br_b, g.nl);
    read_vec(f, g.c2, g.ng);
    read_vec(f, g.c1, g.ng);
    read_vec(f, g.c0, g.ng);
    const rpf::Presolve P = rpf::build_presolve(g);
    check_global(P);
    check_packs(P);
    const rpf::PresolveStats s = rpf::stats(P);
    std::printf("%d %d %d %lld %lld %lld %lld %lld %lld %lld %lld %lld\n", P.nx, P.nu, P.m, (long long)s.nnz_lu,
                (long long)s.nlev_lo, (long long)s.nlev_up, (long long)s.npacks, (long long)s.ntop,
                (long long)s.max_tail_fwd_levels, (long long)s.max_tail_bwd_levels, (long long)s.tail_rows,
                (long long)s.refactor_updates);
  } catch (const std::exception& e) {
    std::fprintf(stderr, "presolve check failed: %s\n", e.what());
    return 1;
  }
  return 0;
}
