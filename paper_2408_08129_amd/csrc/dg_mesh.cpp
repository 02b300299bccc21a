// Host-side forest mesh: base grid refined by rules on logical cell centres (Section 3.1, Fig. 1:
// refinement near the orography in both horizontal and vertical directions), 2:1 balance check,
// face classification (wall / conforming / fine side / coarse side of a hanging face) and Morton
// ordering of the leaves.  Neighbours are found through a hash map keyed by (level, index).
#include "dg_mesh.hpp"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace dg {

static inline uint64_t key_of(int lev, int i0, int i1, int i2) {
  return ((uint64_t)lev << 60) | ((uint64_t)(uint32_t)i0 << 40) | ((uint64_t)(uint32_t)i1 << 20) |
         (uint64_t)(uint32_t)i2;
}

static inline uint64_t spread3(uint64_t v) {  // 20 bits -> every third bit
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}
static inline uint64_t spread2(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 31; ++b) r |= ((v >> b) & 1ull) << (2 * b);
  return r;
}

int build_mesh(const dg_case_desc& cs, int degree, HostMesh& M, std::string& err) {
  if (cs.dim != 2 && cs.dim != 3) { err = "dim must be 2 or 3"; return DG_EINVAL; }
  if (degree < 1 || degree > 5) { err = "degree must be in [1, 5]"; return DG_EUNSUPPORTED; }
  if (cs.n_rules < 0 || cs.n_rules > DG_MAX_RULES) { err = "n_rules out of range"; return DG_EINVAL; }
  const int D = cs.dim;
  M.dim = D;
  M.degree = degree;
  M.np = degree + 1;
  M.nloc = 1;
  for (int a = 0; a < D; ++a) M.nloc *= M.np;
  for (int a = 0; a < 3; ++a) { M.nb[a] = 1; M.L[a] = 1.0; M.per[a] = 0; }
  for (int a = 0; a < D; ++a) {
    const int da = (D == 3) ? a : (a == 0 ? 0 : 2);
    M.nb[a] = cs.nbase[da];
    M.L[a] = cs.length[da];
    if (M.nb[a] < 1 || !(M.L[a] > 0.0)) { err = "bad base grid or extent"; return DG_EINVAL; }
  }
  M.per[0] = cs.periodic_x ? 1 : 0;
  if (D == 3) M.per[1] = cs.periodic_y ? 1 : 0;
  const double H = M.L[D - 1];

  struct Rec { int lev; int i[3]; };
  std::vector<Rec> cur, next, leaves;
  cur.reserve((size_t)M.nb[0] * M.nb[1] * (D == 3 ? M.nb[2] : 1));
  for (int k2 = 0; k2 < (D == 3 ? M.nb[2] : 1); ++k2)
    for (int k1 = 0; k1 < M.nb[1]; ++k1)
      for (int k0 = 0; k0 < M.nb[0]; ++k0) cur.push_back(Rec{0, {k0, k1, D == 3 ? k2 : 0}});
  for (int lev = 0; !cur.empty(); ++lev) {
    next.clear();
    for (const Rec& c : cur) {
      bool refine = false;
      if (lev < cs.n_rules) {
        const dg_refine_rule& ru = cs.rules[lev];
        double ctr[3];
        for (int a = 0; a < D; ++a) ctr[a] = M.L[a] * (c.i[a] + 0.5) / ((double)M.nb[a] * (1 << lev));
        refine = ctr[D - 1] < ru.zeta_max;
        if (refine && ru.half_width_x > 0.0) refine = std::fabs(ctr[0] - ru.x_c) < ru.half_width_x;
        if (refine && D == 3 && ru.half_width_y > 0.0) refine = std::fabs(ctr[1] - ru.y_c) < ru.half_width_y;
      }
      if (!refine) { leaves.push_back(c); continue; }
      for (int ch = 0; ch < (1 << D); ++ch) {
        Rec r{lev + 1, {0, 0, 0}};
        for (int a = 0; a < D; ++a) r.i[a] = 2 * c.i[a] + ((ch >> a) & 1);
        next.push_back(r);
      }
    }
    cur.swap(next);
  }
  int lmax = 0;
  for (const Rec& r : leaves) lmax = std::max(lmax, r.lev);
  M.lmax = lmax;
  for (int a = 0; a < D; ++a)
    if (((long)M.nb[a] << lmax) >= (1L << 20)) { err = "mesh too fine for 20-bit indices"; return DG_EINVAL; }

  // Morton order of the finest-level anchors
  std::vector<std::pair<uint64_t, int>> order(leaves.size());
  for (size_t c = 0; c < leaves.size(); ++c) {
    const Rec& r = leaves[c];
    const int sh = lmax - r.lev;
    uint64_t key;
    if (D == 3)
      key = spread3((uint64_t)r.i[0] << sh) | (spread3((uint64_t)r.i[1] << sh) << 1) |
            (spread3((uint64_t)r.i[2] << sh) << 2);
    else
      key = spread2((uint64_t)r.i[0] << sh) | (spread2((uint64_t)r.i[1] << sh) << 1);
    order[c] = {key, (int)c};
  }
  std::sort(order.begin(), order.end());
  const int nc = (int)leaves.size();
  M.ncell = nc;
  M.cell.assign((size_t)4 * nc, 0);
  std::unordered_map<uint64_t, int> where;
  where.reserve((size_t)nc * 2);
  for (int c = 0; c < nc; ++c) {
    const Rec& r = leaves[order[c].second];
    M.cell[4 * c] = r.lev;
    for (int a = 0; a < 3; ++a) M.cell[4 * c + 1 + a] = r.i[a];
    where[key_of(r.lev, r.i[0], r.i[1], r.i[2])] = c;
  }

  const int NF = 2 * D;
  M.fkind.assign((size_t)NF * nc, 0);
  M.fnbr.assign((size_t)4 * NF * nc, -1);
  M.nhang = 0;
  auto find = [&](int lev, const int* i) -> int {
    auto it = where.find(key_of(lev, i[0], i[1], i[2]));
    return it == where.end() ? -1 : it->second;
  };
  for (int c = 0; c < nc; ++c) {
    const int lev = M.cell[4 * c];
    const int* ci = &M.cell[4 * c + 1];
    for (int k = 0; k < D; ++k)
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * k + s;
        int* kind = &M.fkind[(size_t)NF * c + f];
        int* nb = &M.fnbr[((size_t)NF * c + f) * 4];
        int j[3] = {ci[0], ci[1], ci[2]};
        j[k] += s ? 1 : -1;
        const int nk = M.nb[k] << lev;
        if (j[k] < 0 || j[k] >= nk) {
          if (!M.per[k]) { *kind = kWall; continue; }
          j[k] = (j[k] + nk) % nk;
        }
        int o = find(lev, j);
        if (o >= 0) { *kind = kConf; nb[0] = o; continue; }
        if (lev > 0) {
          int jp[3] = {j[0] >> 1, j[1] >> 1, j[2] >> 1};
          if (D == 2) jp[2] = 0;
          o = find(lev - 1, jp);
          if (o >= 0) { *kind = kFine; nb[0] = o; continue; }
        }
        // finer neighbours: the 2^(d-1) children of the same-level neighbour touching this face
        bool ok = true;
        for (int sub = 0; sub < (1 << (D - 1)); ++sub) {
          int jc[3] = {0, 0, 0};
          int t = 0;
          for (int a = 0; a < D; ++a) {
            if (a == k) jc[a] = 2 * j[a] + (s ? 0 : 1);
            else { jc[a] = 2 * j[a] + ((sub >> t) & 1); ++t; }
          }
          const int oc = find(lev + 1, jc);
          if (oc < 0) { ok = false; break; }
          nb[sub] = oc;
        }
        if (!ok) {
          err = "mesh violates 2:1 balance across a face";
          return DG_EINVAL;
        }
        *kind = kCoarse;
        M.nhang += 1 << (D - 1);
      }
  }
  return DG_OK;
}

}  // namespace dg
