// Host-side setup: validation, partition maps, orderings, symbolic
// factorisation, level schedules and contribution lists (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <queue>
#include <set>
#include <sstream>
#include <unordered_map>

namespace mase {

namespace {

constexpr int VM = 0, PINJ = 1, QINJ = 2, PF = 3, QF = 4, QT = 6;

int32_t round_up(int64_t v, int64_t m) { return (int32_t)((v + m - 1) / m * m); }

// A support entry of a row: (role, local bus).
struct Sup { int role, bus; };

// Minimum-degree elimination of nodes [0, nelim) of a graph on nn nodes
// (nodes >= nelim are never eliminated).  Ties go to the smaller index.
// Returns the elimination order and each eliminated node's neighbours at
// the moment it is eliminated (its column structure in the factor).
void min_degree(int nn, int nelim, std::vector<std::set<int>> adj, std::vector<int>& order,
                std::vector<std::vector<int>>& nbrs_at) {
  using P = std::pair<int, int>;
  std::priority_queue<P, std::vector<P>, std::greater<P>> pq;
  std::vector<char> done(nn, 0);
  for (int v = 0; v < nelim; ++v) pq.push({(int)adj[v].size(), v});
  order.clear();
  nbrs_at.assign(nn, {});
  while (!pq.empty()) {
    auto [d, v] = pq.top();
    pq.pop();
    if (done[v] || d != (int)adj[v].size()) continue;
    done[v] = 1;
    order.push_back(v);
    std::vector<int> nb(adj[v].begin(), adj[v].end());
    nbrs_at[v] = nb;
    for (int a : nb) adj[a].erase(v);
    for (int a : nb) {
      for (int b : nb)
        if (b != a) adj[a].insert(b);
      if (a < nelim && !done[a]) pq.push({(int)adj[a].size(), a});
    }
  }
}

// Relabels a system after ordering: eliminated nodes take their elimination
// positions, the rest keep their relative order after them.  Fills gbus,
// strct and returns old->new.
std::vector<int> relabel(SysPlan& s, const std::vector<int>& gbus_old, int nelim,
                         const std::vector<int>& order,
                         const std::vector<std::vector<int>>& nbrs_at) {
  const int nn = (int)gbus_old.size();
  std::vector<int> newof(nn, -1);
  int c = 0;
  for (int v : order) newof[v] = c++;
  for (int v = nelim; v < nn; ++v) newof[v] = c++;
  s.nn = nn;
  s.gbus.assign(nn, -1);
  for (int v = 0; v < nn; ++v) s.gbus[newof[v]] = gbus_old[v];
  s.strct.assign(nn, {});
  for (int v : order) {
    auto& st = s.strct[newof[v]];
    for (int a : nbrs_at[v]) st.push_back(newof[a]);
    std::sort(st.begin(), st.end());
  }
  return newof;
}

// Packed offsets, levels and the level schedule of a system whose nn, ne,
// gbus and strct are set.
void finish_system(SysPlan& s, int bs_threads) {
  s.nt = s.nn - s.ne;
  s.col_off.assign(s.ne, 0);
  int64_t cur = 0;
  for (int j = 0; j < s.ne; ++j) {
    s.col_off[j] = (int32_t)cur;
    cur += 4 * (1 + (int64_t)s.strct[j].size());
  }
  cur = round_up(cur, 16);
  s.tail_off = (int32_t)cur;
  s.ld = round_up(2 * (int64_t)s.nt, 16);
  cur += s.packed_tail ? 2 * (int64_t)s.nt * (s.nt + 1) : (int64_t)s.ld * s.ld;
  if (cur > (int64_t)1 << 30) throw std::runtime_error("system too large for 32-bit offsets");
  s.nval = (int32_t)cur;

  // elimination tree levels (leaves at 0)
  s.level.assign(s.ne, 0);
  for (int j = 0; j < s.ne; ++j) {
    int par = -1;
    for (int i : s.strct[j])
      if (i < s.ne) { par = i; break; }
    if (par >= 0) s.level[par] = std::max(s.level[par], s.level[j] + 1);
  }
  int ntree = 0;
  for (int j = 0; j < s.ne; ++j) ntree = std::max(ntree, s.level[j] + 1);
  std::vector<std::vector<int>> tree_lev(ntree);
  for (int j = 0; j < s.ne; ++j) tree_lev[s.level[j]].push_back(j);
  // Schedule steps: the columns of one tree level are independent, so a wide
  // level is split into consecutive steps whose LDS staging (4 doubles per
  // factor block, 2 per y_j) stays within the budget.
  std::vector<std::vector<int>> bylev;
  for (const auto& cols : tree_lev) {
    std::vector<int> cur;
    int need = 0;
    for (int j : cols) {
      const int add = 4 * (int)s.strct[j].size() + 2;
      if (!cur.empty() && need + add > LDS_STAGE_DOUBLES) {
        bylev.push_back(cur);
        cur.clear();
        need = 0;
      }
      cur.push_back(j);
      need += add;
    }
    if (!cur.empty()) bylev.push_back(cur);
  }
  s.nlev = (int)bylev.size();

  s.cd_ptr.assign(1, 0);
  s.up_ptr.assign(1, 0);
  s.rb_ptr.assign(1, 0);
  s.bs_ptr.assign(1, 0);
  s.cd_items.clear(); s.up_tgt.clear(); s.up_con.clear();
  s.rb_tgt.clear(); s.rb_con.clear(); s.bs_items.clear(); s.bs_con.clear();
  s.up_tgt_img.clear(); s.up_con_img.clear(); s.rb_con_img.clear();
  // lij / lpj: LDS staging slots of the level's factor blocks; oij / opj:
  // the same blocks' offsets in the packed storage (for the variant that
  // keeps the whole system in LDS and needs no staging)
  struct UpT { int32_t tgt, stride, lij, lpj, j, oij, opj; };
  struct RbT { int32_t rhs_i, lij, rhs_j, j, oij; };
  s.lds_doubles = 0;
  for (int lev = 0; lev < s.nlev; ++lev) {
    std::vector<UpT> ups;
    std::vector<RbT> rbs;
    // LDS staging of the level: every off-diagonal factor block L_ij of the
    // level's columns gets 4 doubles, then every y_j gets 2 doubles
    int nsrc = 0;
    for (int j : bylev[lev]) nsrc += (int)s.strct[j].size();
    std::unordered_map<int32_t, int32_t> slot_of;  // global block offset -> LDS double offset
    int next_src = 0, next_y = 0;
    std::vector<int32_t> yslot(bylev[lev].size());
    for (size_t q = 0; q < bylev[lev].size(); ++q) {
      const int j = bylev[lev][q];
      yslot[q] = 4 * nsrc + 2 * next_y++;
      s.cd_items.push_back({s.col_off[j], -1, 2 * j, yslot[q]});
      for (int i : s.strct[j]) {
        const int32_t off = s.blk_off(i, j);
        slot_of[off] = 4 * next_src++;
        s.cd_items.push_back({s.col_off[j], off, 0, slot_of[off]});
      }
    }
    s.lds_doubles = std::max(s.lds_doubles, 4 * nsrc + 2 * next_y);
    for (size_t q = 0; q < bylev[lev].size(); ++q) {
      const int j = bylev[lev][q];
      const auto& st = s.strct[j];
      for (size_t a = 0; a < st.size(); ++a) {
        const int i = st[a];
        rbs.push_back({2 * i, slot_of.at(s.blk_off(i, j)), yslot[q], j, s.blk_off(i, j)});
        for (size_t b = 0; b <= a; ++b) {
          const int p = st[b];  // p <= i
          ups.push_back({s.blk_off(i, p), s.blk_stride(i, p), slot_of.at(s.blk_off(i, j)),
                         slot_of.at(s.blk_off(p, j)), j, s.blk_off(i, j), s.blk_off(p, j)});
        }
      }
      // back-solve item for column j
      s.bs_items.push_back({s.col_off[j], 2 * j, (int32_t)s.bs_con.size(),
                            (int32_t)(s.bs_con.size() + st.size())});
      for (int i : st) s.bs_con.push_back({s.blk_off(i, j), 2 * i});
    }
    std::stable_sort(ups.begin(), ups.end(), [](const UpT& a, const UpT& b) {
      return a.tgt != b.tgt ? a.tgt < b.tgt : a.j < b.j;
    });
    for (size_t a = 0; a < ups.size();) {
      size_t b = a;
      while (b < ups.size() && ups[b].tgt == ups[a].tgt) ++b;
      if (b - a == 1) {
        // one contribution: its two LDS slots ride in the target record
        s.up_tgt.push_back({ups[a].tgt, ups[a].stride | UP_SINGLE, ups[a].lij, ups[a].lpj});
        s.up_tgt_img.push_back({ups[a].tgt, ups[a].stride | UP_SINGLE, ups[a].oij, ups[a].opj});
      } else {
        s.up_tgt.push_back({ups[a].tgt, ups[a].stride, (int32_t)s.up_con.size(),
                            (int32_t)(s.up_con.size() + (b - a))});
        s.up_tgt_img.push_back(s.up_tgt.back());
        for (size_t c = a; c < b; ++c) {
          s.up_con.push_back({ups[c].lij, ups[c].lpj});
          s.up_con_img.push_back({ups[c].oij, ups[c].opj});
        }
      }
      a = b;
    }
    std::stable_sort(rbs.begin(), rbs.end(), [](const RbT& a, const RbT& b) {
      return a.rhs_i != b.rhs_i ? a.rhs_i < b.rhs_i : a.j < b.j;
    });
    for (size_t a = 0; a < rbs.size();) {
      size_t b = a;
      while (b < rbs.size() && rbs[b].rhs_i == rbs[a].rhs_i) ++b;
      s.rb_tgt.push_back({rbs[a].rhs_i, (int32_t)s.rb_con.size(),
                          (int32_t)(s.rb_con.size() + (b - a)), 0});
      for (size_t c = a; c < b; ++c) {
        s.rb_con.push_back({rbs[c].lij, rbs[c].rhs_j});
        s.rb_con_img.push_back({rbs[c].oij, 2 * rbs[c].j});
      }
      a = b;
    }
    s.cd_ptr.push_back((int32_t)s.cd_items.size());
    s.up_ptr.push_back((int32_t)s.up_tgt.size());
    s.rb_ptr.push_back((int32_t)s.rb_tgt.size());
    s.bs_ptr.push_back((int32_t)s.bs_items.size());
  }
  // back substitution lane groups: with G lanes per column a level takes
  // ceil(items / (threads / G)) passes, each a round trip for its item
  // records and two (record, then factor block) per step along the longest
  // column, ceil(longest column / G) steps; the cheapest G wins, ties to the
  // larger G
  s.bs_lg.assign(s.nlev + 1, 0);
  for (int lev = 0; lev < s.nlev; ++lev) {
    const int n = s.bs_ptr[lev + 1] - s.bs_ptr[lev];
    int m = 0;
    for (int it = s.bs_ptr[lev]; it < s.bs_ptr[lev + 1]; ++it)
      m = std::max(m, s.bs_items[it].w - s.bs_items[it].z);
    int best = -1;
    int64_t best_cost = 0;
    for (int lg = 0; (1 << lg) <= 64 && (1 << lg) <= bs_threads; ++lg) {
      const int G = 1 << lg, per = bs_threads / G;
      const int64_t cost = (int64_t)((n + per - 1) / per) * (1 + 2 * std::max(1, (m + G - 1) / G));
      if (best < 0 || cost <= best_cost) { best = lg; best_cost = cost; }
    }
    s.bs_lg[lev] = best;
  }
}

std::string check_input(const Input& in) {
  std::ostringstream e;
  if (in.n_bus < 2) return "n_bus must be >= 2";
  if (in.n_branch < 1) return "n_branch must be >= 1";
  if (in.n_area < 1) return "n_area must be >= 1";
  if (in.n_meas < 1) return "n_meas must be >= 1";
  if (in.n_snap < 1) return "n_snap must be >= 1";
  if (in.slack < 0 || in.slack >= in.n_bus) return "slack_bus out of range";
  if (!in.br_from || !in.br_to || !in.br_r || !in.br_x || !in.br_b || !in.bus_area ||
      !in.meas_type || !in.meas_at || !in.meas_sigma)
    return "null input array";
  for (int e2 = 0; e2 < in.n_branch; ++e2) {
    const int f = in.br_from[e2], t = in.br_to[e2];
    if (f < 0 || f >= in.n_bus || t < 0 || t >= in.n_bus) {
      e << "branch " << e2 << " bus index out of range";
      return e.str();
    }
    if (f == t) { e << "branch " << e2 << " connects a bus to itself"; return e.str(); }
    const double r = in.br_r[e2], x = in.br_x[e2], b = in.br_b[e2];
    if (!std::isfinite(r) || !std::isfinite(x) || !std::isfinite(b) || r * r + x * x <= 0.0) {
      e << "branch " << e2 << " has a non-finite or zero impedance";
      return e.str();
    }
  }
  for (int b = 0; b < in.n_bus; ++b)
    if (in.bus_area[b] < 0 || in.bus_area[b] >= in.n_area) {
      e << "bus " << b << " area out of range";
      return e.str();
    }
  for (int i = 0; i < in.n_meas; ++i) {
    const int ty = in.meas_type[i], at = in.meas_at[i];
    if (ty < VM || ty > QT) { e << "measurement " << i << " has an unknown type"; return e.str(); }
    const int lim = ty <= QINJ ? in.n_bus : in.n_branch;
    if (at < 0 || at >= lim) { e << "measurement " << i << " location out of range"; return e.str(); }
    const double s = in.meas_sigma[i];
    if (!(s > 0.0) || !std::isfinite(s)) { e << "measurement " << i << " sigma must be > 0"; return e.str(); }
  }
  if (in.gamma_mode != 0 && in.gamma_mode != 1) return "unknown gamma_mode";
  return "";
}

}  // namespace

int32_t SysPlan::blk_off(int i, int j) const {
  if (j < ne) {
    if (i == j) return col_off[j];
    const auto& s = strct[j];
    auto it = std::lower_bound(s.begin(), s.end(), i);
    if (it == s.end() || *it != i) throw std::logic_error("block not in pattern");
    return col_off[j] + 4 * (1 + (int32_t)(it - s.begin()));
  }
  const int a = i - ne, b = j - ne;
  if (packed_tail) return tail_off + 4 * (b * nt - b * (b - 1) / 2 + (a - b));
  return tail_off + 2 * b * ld + 2 * a;
}

int32_t SysPlan::blk_stride(int /*i*/, int j) const { return (j < ne || packed_tail) ? 2 : ld; }

void SysPlan::build_supernodes() {
  sn.clear();
  sn2.clear();
  sn_rows.clear();
  sn_tgt.clear();
  sn_tbase.assign(1, 0);
  sn_lds_bytes = 0;
  int j = 0;
  while (j < ne) {
    int w = 1;
    while (j + w < ne && w < SN_MAX_W) {
      const auto& a = strct[j + w - 1];
      const auto& c = strct[j + w];
      if (a.empty() || a[0] != j + w || a.size() != c.size() + 1) break;
      if (!std::equal(c.begin(), c.end(), a.begin() + 1)) break;
      ++w;
    }
    const auto& R = strct[j + w - 1];
    const int r = (int)R.size();
    const int ntail = (int)(R.end() - std::lower_bound(R.begin(), R.end(), ne));
    sn.push_back({j, w, r, (int32_t)sn_rows.size()});
    sn2.push_back({col_off[j], col_off[j + w - 1] + 4 * (1 + r) - col_off[j], (int32_t)sn_tgt.size(), ntail});
    sn_rows.insert(sn_rows.end(), R.begin(), R.end());
    for (int a = 0; a < r; ++a)
      for (int c = 0; c <= a; ++c) sn_tgt.push_back(blk_off(R[a], R[c]));
    sn_tbase.push_back((int32_t)sn_tgt.size());
    sn_lds_bytes = std::max(sn_lds_bytes, sn_lds_bytes_of(w, r));
    j += w;
  }
  // subtree roots, in supernode order (children before parents)
  const int nsn = (int)sn.size();
  std::vector<int> sn_of(ne, -1);
  for (int q = 0; q < nsn; ++q)
    for (int b = 0; b < sn[q].y; ++b) sn_of[sn[q].x + b] = q;
  sn_root.assign(nsn, -1);
  sn_cost.assign(nsn, 0.0);
  for (int q = nsn - 1; q >= 0; --q) {
    const int r = sn[q].z;
    const int first = r ? sn_rows[sn[q].w] : -1;
    sn_root[q] = (first < 0 || first >= ne) ? q : sn_root[sn_of[first]];
    // per 16-column step: one wave-level 16x16 Cholesky plus row-tile work,
    // then staging, Schur update and write-back in proportion to the rows
    const int Wp = sn_cols_padded(sn[q].y), M = sn_rows_padded(sn[q].y, r);
    sn_cost[q] = (Wp / 16) * (7.0 + 0.6 * M / 16) + 1.5 * M / 16;
  }
  // tail contributions: U_q and c_q offsets, and per tail entry the list of
  // buffer offsets in supernode order
  sn3.clear();
  tail_ent.clear();
  tail_con.clear();
  tl_doubles = 0;
  const int nv = 2 * nt;
  std::vector<std::vector<int32_t>> mat((size_t)nv * nv), rv(nv);
  for (int q = 0; q < nsn; ++q) {
    const int r = sn[q].z, ntail = sn2[q].w, mt = 2 * ntail, nrs = r - ntail;
    const int32_t* R = sn_rows.data() + sn[q].w;
    if (!ntail) {
      sn3.push_back({0, 0, 0, 0});
      continue;
    }
    const int32_t uoff = tl_doubles;
    tl_doubles += (mt * mt + 31) / 32 * 32;
    const int32_t coff = tl_doubles;
    tl_doubles += (mt + 31) / 32 * 32;
    sn3.push_back({uoff, coff, 0, 0});
    auto var = [&](int a) { return 2 * (R[nrs + a / 2] - ne) + (a & 1); };
    for (int a = 0; a < mt; ++a) {
      rv[var(a)].push_back(coff + a);
      for (int c = 0; c < mt; ++c)
        if (var(a) >= var(c)) mat[(size_t)var(c) * nv + var(a)].push_back(uoff + c * mt + a);
    }
  }
  for (int c = 0; c < nv; ++c)
    for (int a = c; a < nv; ++a) {
      const auto& l = mat[(size_t)c * nv + a];
      if (l.empty()) continue;
      tail_ent.push_back({c * ld + a, 0, (int32_t)tail_con.size(), (int32_t)(tail_con.size() + l.size())});
      tail_con.insert(tail_con.end(), l.begin(), l.end());
    }
  for (int a = 0; a < nv; ++a) {
    if (rv[a].empty()) continue;
    tail_ent.push_back({a, 1, (int32_t)tail_con.size(), (int32_t)(tail_con.size() + rv[a].size())});
    tail_con.insert(tail_con.end(), rv[a].begin(), rv[a].end());
  }
  group_supernodes(1);
}

void SysPlan::group_supernodes(int max_groups) {
  const int nsn = (int)sn.size();
  std::vector<int> roots;
  std::vector<double> tree(nsn, 0.0);
  for (int q = 0; q < nsn; ++q) {
    tree[sn_root[q]] += sn_cost[q];
    if (sn_root[q] == q) roots.push_back(q);
  }
  const int G = std::max(1, std::min(max_groups, (int)roots.size()));
  // longest subtree first, each to the group with the least work so far
  std::stable_sort(roots.begin(), roots.end(), [&](int a, int b) { return tree[a] > tree[b]; });
  std::vector<double> load(G, 0.0);
  std::vector<int> grp_of(nsn, 0);
  for (int rt : roots) {
    const int gi = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[gi] += tree[rt];
    grp_of[rt] = gi;
  }
  sn_grp_ptr.assign(G + 1, 0);
  sn_grp.clear();
  for (int gi = 0; gi < G; ++gi) {
    for (int q = 0; q < nsn; ++q)
      if (grp_of[sn_root[q]] == gi) sn_grp.push_back(q);
    sn_grp_ptr[gi + 1] = (int32_t)sn_grp.size();
  }
}

double SysPlan::elim_flops() const {
  double f = 0;
  for (int j = 0; j < ne; ++j) {
    const double r = (double)strct[j].size();
    f += 12 + 14 * r;              // 2x2 Cholesky, block solves, rhs
    f += 16.0 * r * (r + 1) / 2;   // trailing block updates
    f += 8 * r + 8;                // rhs updates
    f += 8 * r + 10;               // back substitution
  }
  return f;
}

int Plan::max_levels() const {
  int m = 0;
  for (int k = 0; k < n_area; ++k) m = std::max(m, sys[k].nlev);
  return m;
}

double Plan::flops_local() const {
  double f = 0;
  for (int k = 0; k < n_area; ++k) f += sys[k].elim_flops();
  return f;
}

double Plan::flops_gamma() const {
  return sys[n_area].elim_flops() + flops_dense();
}

double Plan::bytes_assembly() const {
  double b = 8.0 * n_meas + 16.0 * n_bus;  // z, x
  double tmpl = 0;
  for (int k = 0; k < n_area; ++k) {
    const auto& t = tpl[k];
    // packed G: the 2x2 blocks that some measurement row contributes to
    // (fill positions of the factor are not part of G), b, J
    int64_t nz = 0;
    for (const I4& sl : t.slot) nz += sl.w > sl.z;
    b += 8.0 * 4 * nz + 16.0 * sys[k].nn + 8.0;
    tmpl += 16.0 * t.slot.size() + 8.0 * t.scon.size() + 8.0 * t.rslot.size() + 8.0 * t.rcon.size() +
            12.0 * t.row_type.size() + 40.0 * t.br_lf.size() + 4.0 * (t.inc_ptr.size() + t.inc_end.size());
  }
  tmpl += 8.0 * n_meas;  // weights
  return b + tmpl / std::max(1, n_snap);
}

double Plan::bytes_condense(bool lds) const {
  double b = 0;
  for (int k = 0; k < n_area; ++k) {
    const SysPlan& s = sys[k];
    if (lds && tpl[k].lds_split > 0) {
      // read the compact G (and the Schur block kept in HBM, read and
      // written), write the packed storage once, rhs in and out
      const double in_hbm = (double)(s.nval - tpl[k].lds_split);
      b += 8.0 * 4 * tpl[k].cimg.size() + 8.0 * tpl[k].lds_split + 2.0 * 8 * in_hbm + 2.0 * 16 * s.nn;
    } else {
      b += 2.0 * 8 * s.nval + 2.0 * 16 * s.nn;
    }
  }
  return b;
}

double Plan::bytes_backsolve() const {
  // the areas' back substitution (the boundary system's has its own kernels)
  double b = 0;
  for (int k = 0; k < n_area; ++k) b += 8.0 * sys[k].tail_off + 2.0 * 16 * sys[k].nn;
  return b;
}

double Plan::flops_dense() const {
  // Cholesky and two triangular solves of the dense block's 2 nt variables
  // (its storage is padded to ld; the padding is not counted)
  const double nd = 2.0 * sys[n_area].nt;
  return nd * nd * nd / 3.0 + 2.0 * nd * nd;
}

int Plan::n_gamma_vars() const {
  int n = 0;
  for (int b : gamma_bus) n += (b == slack) ? 1 : 2;
  return n;
}

std::string build_plan(const Input& in, Plan& p) {
  std::string err = check_input(in);
  if (!err.empty()) return err;
  p = Plan();
  p.n_bus = in.n_bus; p.n_branch = in.n_branch; p.n_area = in.n_area;
  p.n_meas = in.n_meas; p.slack = in.slack; p.n_snap = in.n_snap;
  p.br_from.assign(in.br_from, in.br_from + in.n_branch);
  p.br_to.assign(in.br_to, in.br_to + in.n_branch);
  p.sigma.assign(in.meas_sigma, in.meas_sigma + in.n_meas);
  p.bus_area.assign(in.bus_area, in.bus_area + in.n_bus);
  const int N = in.n_bus, B = in.n_branch, K = in.n_area;
  const auto& area = p.bus_area;
  const auto& F = p.br_from;
  const auto& T = p.br_to;

  // boundary buses: terminals of cut branches (Section 2.3)
  p.is_bnd.assign(N, 0);
  for (int e = 0; e < B; ++e)
    if (area[F[e]] != area[T[e]]) p.is_bnd[F[e]] = p.is_bnd[T[e]] = 1;
  p.gamma_canon_pos.assign(N, -1);
  for (int b = 0; b < N; ++b)
    if (p.is_bnd[b]) {
      p.gamma_canon_pos[b] = (int32_t)p.gamma_bus.size();
      p.gamma_bus.push_back(b);
    }

  // adjacency (for connectivity and injections)
  std::vector<std::vector<int>> inc(N);  // incident branches
  for (int e = 0; e < B; ++e) { inc[F[e]].push_back(e); inc[T[e]].push_back(e); }

  // each area: non-empty, connected, with an internal bus
  {
    std::vector<int> seen(N, 0), cnt(K, 0), inter(K, 0);
    for (int b = 0; b < N; ++b) { cnt[area[b]]++; if (!p.is_bnd[b]) inter[area[b]]++; }
    for (int k = 0; k < K; ++k) {
      if (cnt[k] == 0) return "area " + std::to_string(k) + " has no bus";
      if (inter[k] == 0) return "area " + std::to_string(k) + " has no internal bus";
    }
    std::vector<int> reached(K, 0);
    for (int b = 0; b < N; ++b) {
      if (seen[b]) continue;
      const int k = area[b];
      if (reached[k]) return "area " + std::to_string(k) + " is not connected";
      reached[k] = 1;
      std::vector<int> stack{b};
      seen[b] = 1;
      while (!stack.empty()) {
        int u = stack.back(); stack.pop_back();
        for (int e : inc[u]) {
          int v = F[e] == u ? T[e] : F[e];
          if (area[v] == k && !seen[v]) { seen[v] = 1; stack.push_back(v); }
        }
      }
    }
  }

  // measurement ownership
  p.meas_area.assign(in.n_meas, 0);
  for (int i = 0; i < in.n_meas; ++i) {
    const int ty = in.meas_type[i], at = in.meas_at[i];
    if (ty <= QINJ) p.meas_area[i] = area[at];
    else if (ty == PF || ty == QF) p.meas_area[i] = area[F[at]];
    else p.meas_area[i] = area[T[at]];
  }
  std::vector<std::vector<int>> rows_of(K);
  for (int i = 0; i < in.n_meas; ++i) rows_of[p.meas_area[i]].push_back(i);

  p.sys.assign(K + 1, SysPlan());
  p.tpl.assign(K, AreaTemplates());
  p.local_of_bus.assign(K, std::vector<int32_t>(N, -1));

  // ---------------- areas ----------------
  for (int k = 0; k < K; ++k) {
    std::vector<int> internal, tail;
    std::set<int> tailset;
    for (int b = 0; b < N; ++b)
      if (area[b] == k) {
        if (p.is_bnd[b]) tailset.insert(b);
        else internal.push_back(b);
      }
    std::vector<int> lbr;  // local branches: at least one end in area k
    for (int e = 0; e < B; ++e)
      if (area[F[e]] == k || area[T[e]] == k) {
        lbr.push_back(e);
        if (area[F[e]] != area[T[e]]) { tailset.insert(F[e]); tailset.insert(T[e]); }
      }
    if (lbr.size() > (size_t)MAX_LOCAL_BRANCH) return "too many branches in one area";
    tail.assign(tailset.begin(), tailset.end());
    const int ni = (int)internal.size();
    std::vector<int> gold(internal);
    gold.insert(gold.end(), tail.begin(), tail.end());
    const int nn = (int)gold.size();
    auto& lob = p.local_of_bus[k];
    for (int v = 0; v < nn; ++v) lob[gold[v]] = v;
    std::unordered_map<int, int> lbr_of;
    for (size_t a = 0; a < lbr.size(); ++a) lbr_of[lbr[a]] = (int)a;

    // row supports in initial local indices
    const auto& rows = rows_of[k];
    std::vector<std::vector<Sup>> sup(rows.size());
    for (size_t r = 0; r < rows.size(); ++r) {
      const int i = rows[r], ty = in.meas_type[i], at = in.meas_at[i];
      if (ty == VM) {
        sup[r].push_back({ROLE_SELF, lob[at]});
      } else if (ty == PINJ || ty == QINJ) {
        sup[r].push_back({ROLE_SELF, lob[at]});
        for (int e : inc[at]) {
          const int o = F[e] == at ? T[e] : F[e];
          sup[r].push_back({lbr_of.at(e), lob[o]});
        }
      } else {
        const bool from = (ty == PF || ty == QF);
        const int a = from ? F[at] : T[at], o = from ? T[at] : F[at];
        sup[r].push_back({ROLE_SELF, lob[a]});
        sup[r].push_back({ROLE_OTHER, lob[o]});
      }
    }
    // bus-level pattern and minimum-degree order of the internal buses
    std::vector<std::set<int>> adj(nn);
    for (auto& s : sup)
      for (auto& a : s)
        for (auto& b : s)
          if (a.bus != b.bus) adj[a.bus].insert(b.bus);
    std::vector<int> order;
    std::vector<std::vector<int>> nbrs_at;
    min_degree(nn, ni, adj, order, nbrs_at);
    if ((int)order.size() != ni) return "ordering failed";
    SysPlan& s = p.sys[k];
    std::vector<int> newof = relabel(s, gold, ni, order, nbrs_at);
    s.ne = ni;
    for (int v = 0; v < nn; ++v) lob[gold[v]] = newof[v];
    for (auto& sv : sup)
      for (auto& a : sv) a.bus = newof[a.bus];
    s.packed_tail = true;
    try { finish_system(s, BS_THREADS_AREA); } catch (std::exception& ex) { return ex.what(); }
    if (p.slack >= 0 && area[p.slack] == k && !p.is_bnd[p.slack]) s.pin_off = s.col_off[lob[p.slack]];

    // templates
    AreaTemplates& t = p.tpl[k];
    for (int e : lbr) {
      t.br_gid.push_back(e);
      t.br_lf.push_back(lob[F[e]]);
      t.br_lt.push_back(lob[T[e]]);
      const double r = in.br_r[e], x = in.br_x[e], z2 = r * r + x * x;
      t.br_g.push_back(r / z2);
      t.br_bs.push_back(-x / z2);
      t.br_hb.push_back(0.5 * in.br_b[e]);
    }
    t.inc_ptr.assign(nn + 1, 0);
    for (int v = 0; v < nn; ++v) {
      const int b = s.gbus[v];
      if (area[b] == k)
        for (int e : inc[b]) t.inc_end.push_back((lbr_of.at(e) << 1) | (F[e] == b ? 0 : 1));
      t.inc_ptr[v + 1] = (int32_t)t.inc_end.size();
    }
    for (size_t r = 0; r < rows.size(); ++r) {
      const int i = rows[r], ty = in.meas_type[i], at = in.meas_at[i];
      t.row_type.push_back(ty);
      t.row_loc.push_back(ty <= QINJ ? lob[at] : lbr_of.at(at));
      t.row_meas.push_back(i);
    }
    // G contributions grouped by target block offset
    std::unordered_map<int32_t, std::vector<I2>> by_blk;
    std::vector<std::vector<I2>> by_bus(nn);
    for (size_t r = 0; r < rows.size(); ++r) {
      const auto& sv = sup[r];
      for (const auto& a : sv) {
        by_bus[a.bus].push_back({(int32_t)r, a.role});
        for (const auto& b : sv) {
          if (a.bus < b.bus) continue;  // block (a.bus, b.bus) with row bus >= column bus
          by_blk[s.blk_off(a.bus, b.bus)].push_back({(int32_t)r, a.role | (b.role << 16)});
        }
      }
    }
    auto emit = [&](int i, int j) {
      const int32_t off = s.blk_off(i, j);
      const int32_t cb = (int32_t)t.scon.size();
      auto it = by_blk.find(off);
      if (it != by_blk.end()) for (auto& c : it->second) t.scon.push_back(c);
      const int32_t st = s.blk_stride(i, j);
      t.slot.push_back({off, i == j ? -st : st, cb, (int32_t)t.scon.size()});
    };
    for (int j = 0; j < s.ne; ++j) {
      emit(j, j);
      for (int i : s.strct[j]) emit(i, j);
    }
    for (int q = s.ne; q < nn; ++q)
      for (int pp = q; pp < nn; ++pp) emit(pp, q);
    for (int v = 0; v < nn; ++v) {
      const int32_t cb = (int32_t)t.rcon.size();
      for (auto& c : by_bus[v]) t.rcon.push_back(c);
      t.rslot.push_back({cb, (int32_t)t.rcon.size()});
    }
    // compact output for the elimination in LDS: everything in LDS if it
    // fits beside the rhs, else all but the Schur block (which stays in HBM)
    if ((int64_t)s.nval + 2 * nn <= AREA_LDS_DOUBLES) t.lds_split = s.nval;
    else if ((int64_t)s.tail_off + 2 * nn <= AREA_LDS_DOUBLES) t.lds_split = s.tail_off;
    else t.lds_split = 0;
    for (const I4& sl : t.slot) {
      if (sl.x < t.lds_split) {
        if (sl.w <= sl.z) continue;  // fill: zero in LDS
        t.cslot.push_back({4 * (int32_t)t.cimg.size(), sl.y < 0 ? -2 : 2, sl.z, sl.w});
        t.cimg.push_back(sl.x);
      } else {
        t.tslot.push_back(sl);
      }
    }
  }

  // ---------------- boundary system ----------------
  {
    SysPlan& g = p.sys[K];
    const int nn = (int)p.gamma_bus.size();
    std::vector<int> gold(p.gamma_bus.begin(), p.gamma_bus.end());
    std::vector<std::set<int>> adj(nn);
    for (int k = 0; k < K; ++k) {
      const SysPlan& s = p.sys[k];
      for (int a = s.ne; a < s.nn; ++a)
        for (int b = s.ne; b < s.nn; ++b)
          if (a != b) adj[p.gamma_canon_pos[s.gbus[a]]].insert(p.gamma_canon_pos[s.gbus[b]]);
    }
    if (in.gamma_mode == 0 && nn > 0) {
      std::vector<int> order;
      std::vector<std::vector<int>> nbrs_at;
      min_degree(nn, nn, adj, order, nbrs_at);
      // Elimination-tree levels of the full minimum-degree elimination.  The
      // top levels that hold a single column each form a chain (it includes
      // the root supernode): those columns are eliminated one after another
      // anyway, so they go to the dense trailing block, factored with dense
      // kernels.  The chain is closed under ancestors, so moving it to the
      // end keeps a valid elimination order with the same fill.
      std::vector<int> pos(nn);
      for (int q = 0; q < nn; ++q) pos[order[q]] = q;
      std::vector<int> lev(nn, 0);
      for (int q = 0; q < nn; ++q) {
        int par = nn;
        for (int a : nbrs_at[order[q]]) par = std::min(par, pos[a]);
        if (par < nn) lev[par] = std::max(lev[par], lev[q] + 1);
      }
      int nlev = 0;
      for (int q = 0; q < nn; ++q) nlev = std::max(nlev, lev[q] + 1);
      std::vector<int> cnt(nlev, 0);
      for (int q = 0; q < nn; ++q) cnt[lev[q]]++;
      int cut = nlev;
      while (cut > 0 && cnt[cut - 1] == 1) --cut;
      std::vector<int> elim, tailn;
      for (int q = 0; q < nn; ++q) (lev[q] >= cut ? tailn : elim).push_back(order[q]);
      std::vector<int> newof(nn, -1);
      int c2 = 0;
      for (int v : elim) newof[v] = c2++;
      for (int v : tailn) newof[v] = c2++;
      g.nn = nn;
      g.ne = (int)elim.size();
      g.gbus.assign(nn, -1);
      for (int v = 0; v < nn; ++v) g.gbus[newof[v]] = gold[v];
      g.strct.assign(nn, {});
      for (int v : elim) {
        auto& st = g.strct[newof[v]];
        for (int a : nbrs_at[v]) st.push_back(newof[a]);
        std::sort(st.begin(), st.end());
      }
    } else {
      g.nn = nn;
      g.gbus = gold;
      g.strct.assign(nn, {});
      g.ne = 0;
    }
    try {
      finish_system(g, BS_THREADS_GAMMA);
      g.build_supernodes();
    } catch (std::exception& ex) { return ex.what(); }
    std::vector<int> gpos(N, -1);  // bus -> Gamma local index
    for (int v = 0; v < nn; ++v) gpos[g.gbus[v]] = v;
    if (p.is_bnd[p.slack]) g.pin_off = g.blk_off(gpos[p.slack], gpos[p.slack]);

    // per-snapshot layout
    p.val_off.assign(K + 1, 0);
    p.rhs_off.assign(K + 1, 0);
    int64_t vo = 0, ro = 0;
    for (int k = 0; k <= K; ++k) {
      p.val_off[k] = (int32_t)vo;
      p.rhs_off[k] = (int32_t)ro;
      vo = round_up(vo + p.sys[k].nval, 32);
      ro = round_up(ro + 2 * (int64_t)p.sys[k].nn, 32);
      if (vo > ((int64_t)1 << 31) - 64) return "per-snapshot storage over 2^31 doubles";
    }
    p.lds_areas = false;
    p.gc_off.assign(K, 0);
    for (int k = 0; k < K; ++k) {
      p.gc_off[k] = (int32_t)vo;
      vo = round_up(vo + 4 * (int64_t)p.tpl[k].cimg.size(), 32);
      p.lds_areas |= p.tpl[k].lds_split > 0;
      if (vo > ((int64_t)1 << 31) - 64) return "per-snapshot storage over 2^31 doubles";
    }
    p.vstride = vo;
    p.rstride = ro;

    // Gamma slots: gather from the areas' dense Schur blocks
    std::unordered_map<int32_t, std::vector<I4>> by_blk;
    std::vector<std::vector<int32_t>> rb(nn);
    for (int k = 0; k < K; ++k) {
      const SysPlan& s = p.sys[k];
      for (int a = s.ne; a < s.nn; ++a) {
        const int ga = gpos[s.gbus[a]];
        rb[ga].push_back(p.rhs_off[k] + 2 * a);
        for (int b = s.ne; b <= a; ++b) {
          const int gb = gpos[s.gbus[b]];
          const int32_t src = p.val_off[k] + s.blk_off(a, b);
          const int32_t sst = s.blk_stride(a, b);
          if (ga >= gb) by_blk[g.blk_off(ga, gb)].push_back({src, sst, 0, 0});
          else by_blk[g.blk_off(gb, ga)].push_back({src, sst, 1, 0});
        }
      }
    }
    auto emit = [&](int i, int j) {
      const int32_t off = g.blk_off(i, j);
      const int32_t cb = (int32_t)p.g_con.size();
      auto it = by_blk.find(off);
      if (it != by_blk.end()) for (auto& c : it->second) p.g_con.push_back(c);
      const int32_t st = g.blk_stride(i, j);
      p.g_slot.push_back({off, i == j ? -st : st, cb, (int32_t)p.g_con.size()});
    };
    for (int j = 0; j < g.ne; ++j) {
      emit(j, j);
      for (int i : g.strct[j]) emit(i, j);
    }
    for (int q = g.ne; q < nn; ++q)
      for (int pp = q; pp < nn; ++pp) emit(pp, q);
    for (int v = 0; v < nn; ++v) {
      const int32_t cb = (int32_t)p.g_rcon.size();
      for (int32_t o : rb[v]) p.g_rcon.push_back(o);
      p.g_rslot.push_back({cb, (int32_t)p.g_rcon.size()});
    }

    // scatter-back sources and per-bus dx sources
    p.tail_src_ptr.assign(K + 1, 0);
    for (int k = 0; k < K; ++k) {
      const SysPlan& s = p.sys[k];
      for (int a = s.ne; a < s.nn; ++a) p.tail_src.push_back(p.rhs_off[K] + 2 * gpos[s.gbus[a]]);
      p.tail_src_ptr[k + 1] = (int32_t)p.tail_src.size();
    }
    p.bus_dx_src.assign(N, -1);
    for (int b = 0; b < N; ++b) {
      if (p.is_bnd[b]) p.bus_dx_src[b] = p.rhs_off[K] + 2 * gpos[b];
      else p.bus_dx_src[b] = p.rhs_off[area[b]] + 2 * p.local_of_bus[area[b]][b];
    }
  }

  // launch order: largest elimination work first
  p.area_order.resize(K);
  std::iota(p.area_order.begin(), p.area_order.end(), 0);
  // The area kernels run one workgroup per (area, snapshot), and their time
  // is set by the level elimination's chain of dependent memory round trips:
  // two per level plus two per extra pass over its column items (256 per
  // pass) or update targets (512 per pass).
  std::vector<double> work(K);
  for (int k = 0; k < K; ++k) {
    const SysPlan& s = p.sys[k];
    double rt = 0;
    for (int l = 0; l < s.nlev; ++l) {
      const int items = s.cd_ptr[l + 1] - s.cd_ptr[l], targets = s.up_ptr[l + 1] - s.up_ptr[l];
      rt += 2.0 * ((items + 255) / 256 + (targets + 511) / 512);
    }
    work[k] = rt;
  }
  std::stable_sort(p.area_order.begin(), p.area_order.end(),
                   [&](int a, int b) { return work[a] > work[b]; });
  // With a multiple of 8 areas the kernels give launch position xcd + 8 m to
  // the chiplet xcd (workgroup b runs on chiplet b mod 8), so every chiplet
  // runs K / 8 areas for all snapshots.  Assign areas to chiplets longest
  // first, each to the least loaded chiplet with room, and order each
  // chiplet's areas longest first.
  if (K % 8 == 0) {
    const int per = K / 8;
    std::vector<std::vector<int>> xcd(8);
    std::vector<double> load(8, 0.0);
    for (int k : p.area_order) {
      int best = -1;
      for (int x = 0; x < 8; ++x)
        if ((int)xcd[x].size() < per && (best < 0 || load[x] < load[best])) best = x;
      xcd[best].push_back(k);
      load[best] += work[k];
    }
    for (int x = 0; x < 8; ++x)
      for (int m = 0; m < per; ++m) p.area_order[x + 8 * m] = xcd[x][m];
  }
  return "";
}

// ---------------- canonical exports ----------------

static void push_vars(std::vector<int32_t>& out, int bus, int slack) {
  if (bus != slack) out.push_back(2 * bus);
  out.push_back(2 * bus + 1);
}

std::vector<int32_t> canon_local_vars(const Plan& p, int k) {
  const SysPlan& s = p.sys[k];
  std::vector<int> internal(s.gbus.begin(), s.gbus.begin() + s.ne);
  std::sort(internal.begin(), internal.end());
  std::vector<int32_t> out;
  for (int b : internal) push_vars(out, b, p.slack);
  for (int a = s.ne; a < s.nn; ++a) push_vars(out, s.gbus[a], p.slack);  // tail is ascending
  return out;
}

int canon_n_internal(const Plan& p, int k) {
  const SysPlan& s = p.sys[k];
  int n = 0;
  for (int a = 0; a < s.ne; ++a) n += (s.gbus[a] == p.slack) ? 1 : 2;
  return n;
}

std::vector<int32_t> canon_gamma_vars(const Plan& p) {
  std::vector<int32_t> out;
  for (int b : p.gamma_bus) push_vars(out, b, p.slack);
  return out;
}

std::vector<int32_t> canon_E(const Plan& p, int k) {
  std::vector<int32_t> gv = canon_gamma_vars(p);
  std::unordered_map<int32_t, int32_t> pos;
  for (size_t i = 0; i < gv.size(); ++i) pos[gv[i]] = (int32_t)i;
  const SysPlan& s = p.sys[k];
  std::vector<int32_t> out;
  for (int a = s.ne; a < s.nn; ++a) {
    const int b = s.gbus[a];
    if (b != p.slack) out.push_back(pos.at(2 * b));
    out.push_back(pos.at(2 * b + 1));
  }
  return out;
}

void canon_pattern(const Plan& p, int k, std::vector<int32_t>& rowptr, std::vector<int32_t>& colidx) {
  const std::vector<int32_t> lv = canon_local_vars(p, k);
  std::unordered_map<int32_t, int32_t> pos;
  for (size_t i = 0; i < lv.size(); ++i) pos[lv[i]] = (int32_t)i;
  const SysPlan& s = p.sys[k];
  const AreaTemplates& t = p.tpl[k];
  std::vector<std::set<int32_t>> rowset(lv.size());
  for (size_t r = 0; r < t.row_type.size(); ++r) {
    const int ty = t.row_type[r], loc = t.row_loc[r];
    std::vector<int32_t> vars;
    auto add_bus = [&](int lbus) {
      const int b = s.gbus[lbus];
      if (b != p.slack) vars.push_back(pos.at(2 * b));
      vars.push_back(pos.at(2 * b + 1));
    };
    if (ty == VM) {
      vars.push_back(pos.at(2 * s.gbus[loc] + 1));
    } else if (ty == PINJ || ty == QINJ) {
      add_bus(loc);
      for (int q = t.inc_ptr[loc]; q < t.inc_ptr[loc + 1]; ++q) {
        const int e = t.inc_end[q] >> 1, side = t.inc_end[q] & 1;
        add_bus(side == 0 ? t.br_lt[e] : t.br_lf[e]);
      }
    } else {
      add_bus(t.br_lf[loc]);
      add_bus(t.br_lt[loc]);
    }
    for (int32_t a : vars)
      for (int32_t b : vars) rowset[a].insert(b);
  }
  rowptr.assign(lv.size() + 1, 0);
  colidx.clear();
  for (size_t i = 0; i < lv.size(); ++i) {
    for (int32_t c : rowset[i]) colidx.push_back(c);
    rowptr[i + 1] = (int32_t)colidx.size();
  }
}

}  // namespace mase
