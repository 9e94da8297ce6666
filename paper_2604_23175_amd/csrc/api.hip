// C ABI of the multi-area estimator (include/mase.h): context management,
// device residency of the plan, launch schedules (batched, graph-captured,
// or the plain per-area/per-snapshot schedule), host-side stage reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "dev.hpp"
#include "launch.hpp"
#include "mase.h"
#include "plan.hpp"
#include "ctx.hpp"

using namespace mase;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPTRY(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(MASE_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

}  // namespace



// Fixed device scratch of mase_solve_stream_noalloc: the stream's slot
// tables (3 n_snap + 2 ints) followed by its per-snapshot results
// (2 n_total ints).  Each GPU the library runs on holds one copy until the
// process ends; every no-alloc call on that GPU shares it.  In host code the
// array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
constexpr int64_t NOALLOC_SCRATCH_INTS = int64_t(1) << 20;  // 4 MiB
static __device__ __align__(256) int32_t scratch[NOALLOC_SCRATCH_INTS];

namespace {

template <class T>
int dalloc(mase_ctx* c, size_t n, T** out) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(1, n) * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(MASE_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  c->dallocs.push_back(p);
  *out = static_cast<T*>(p);
  return 0;
}

// Device address of `scratch` on the current device, resolved once per
// device (the caller has made the context's device current).
int scratch_address(int32_t** out) {
  static std::mutex mu;
  static std::vector<int32_t*> per_dev;
  int dev = 0;
  HIPTRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)per_dev.size() <= dev) per_dev.resize(dev + 1, nullptr);
  if (!per_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MASE_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    per_dev[dev] = static_cast<int32_t*>(p);
  }
  *out = per_dev[dev];
  return 0;
}

template <class D, class H>
int upload(mase_ctx* c, const std::vector<H>& v, const D** out) {
  static_assert(sizeof(D) == sizeof(H), "layout mismatch");
  D* p = nullptr;
  int rc = dalloc(c, v.size(), &p);
  if (rc) return rc;
  if (!v.empty()) HIPTRY(hipMemcpy(p, v.data(), v.size() * sizeof(H), hipMemcpyHostToDevice));
  *out = p;
  return 0;
}

// Sparse part of the boundary system: supernodal when its panels fit in LDS,
// else the level-scheduled engine.
hipError_t launch_gamma_sparse(const mase_ctx* c, int s0, int ns, hipStream_t st) {
  if (c->gamma_snode) return launch_gamma_snode(c->d, s0, ns, c->lds_sn, st);
  return launch_eliminate(c->d, c->plan.n_area, 1, s0, ns, c->lds_el_gamma, st);
}

// Back substitution of the same part: supernodal after the supernodal
// elimination, else level by level.
hipError_t launch_gamma_back(const mase_ctx* c, int s0, int ns, hipStream_t st) {
  if (c->gamma_snode) return launch_gamma_snode_back(c->d, s0, ns, c->lds_sn, st);
  return launch_backsolve(c->d, c->plan.n_area, 1, s0, ns, st);
}

void append_rebased(std::vector<int32_t>& dst, const std::vector<int32_t>& src, int32_t base) {
  for (int32_t v : src) dst.push_back(v + base);
}

int upload_plan(mase_ctx* c) {
  const Plan& p = c->plan;
  const int K = p.n_area;
  std::vector<SysMeta> sm(K + 1);
  std::vector<AreaMeta> am(K);
  std::vector<int32_t> gbus, cd_ptr, up_ptr, rb_ptr, bs_ptr, bs_lg;
  std::vector<I4> cd_items, up_tgt, rb_tgt, bs_items, up_tgt_img;
  std::vector<I2> up_con, rb_con, bs_con, up_con_img, rb_con_img;
  // the areas' elimination runs the level engine over HBM; MASE_AREA_LDS=1
  // holds each area that fits in LDS instead (measured slower at the
  // 9241-bus / 32-area workload: an area image of up to 160 KB leaves one
  // workgroup per CU)
  {
    const char* env = getenv("MASE_AREA_LDS");
    c->area_lds = p.lds_areas && env && env[0] == '1';
  }
  for (int i = 0; i <= K; ++i) {
    const SysPlan& s = p.sys[i];
    SysMeta m{};
    m.nn = s.nn; m.ne = s.ne; m.nt = s.nt; m.ld = s.ld;
    m.tail_off = s.tail_off; m.nval = s.nval; m.pin_off = s.pin_off; m.nlev = s.nlev;
    m.val_off = p.val_off[i]; m.rhs_off = p.rhs_off[i];
    m.asm_pin = s.pin_off;
    m.gbus = (int32_t)gbus.size();
    gbus.insert(gbus.end(), s.gbus.begin(), s.gbus.end());
    m.cd_ptr = (int32_t)cd_ptr.size();
    append_rebased(cd_ptr, s.cd_ptr, (int32_t)cd_items.size());
    cd_items.insert(cd_items.end(), s.cd_items.begin(), s.cd_items.end());
    m.up_ptr = (int32_t)up_ptr.size();
    append_rebased(up_ptr, s.up_ptr, (int32_t)up_tgt.size());
    // a single-contribution target carries its two LDS slots inline: not rebased
    for (const I4& t : s.up_tgt) {
      const int32_t base = (t.y & UP_SINGLE) ? 0 : (int32_t)up_con.size();
      up_tgt.push_back({t.x, t.y, t.z + base, t.w + base});
    }
    for (const I4& t : s.up_tgt_img) {
      const int32_t base = (t.y & UP_SINGLE) ? 0 : (int32_t)up_con_img.size();
      up_tgt_img.push_back({t.x, t.y, t.z + base, t.w + base});
    }
    up_con.insert(up_con.end(), s.up_con.begin(), s.up_con.end());
    up_con_img.insert(up_con_img.end(), s.up_con_img.begin(), s.up_con_img.end());
    rb_con_img.insert(rb_con_img.end(), s.rb_con_img.begin(), s.rb_con_img.end());
    m.rb_ptr = (int32_t)rb_ptr.size();
    append_rebased(rb_ptr, s.rb_ptr, (int32_t)rb_tgt.size());
    for (const I4& t : s.rb_tgt)
      rb_tgt.push_back({t.x, t.y + (int32_t)rb_con.size(), t.z + (int32_t)rb_con.size(), 0});
    rb_con.insert(rb_con.end(), s.rb_con.begin(), s.rb_con.end());
    m.bs_ptr = (int32_t)bs_ptr.size();
    append_rebased(bs_ptr, s.bs_ptr, (int32_t)bs_items.size());
    bs_lg.insert(bs_lg.end(), s.bs_lg.begin(), s.bs_lg.end());  // parallel to bs_ptr
    for (const I4& t : s.bs_items)
      bs_items.push_back({t.x, t.y, t.z + (int32_t)bs_con.size(), t.w + (int32_t)bs_con.size()});
    bs_con.insert(bs_con.end(), s.bs_con.begin(), s.bs_con.end());
    sm[i] = m;
  }
  std::vector<int32_t> br_lf, br_lt, inc_ptr, inc_end, row_type, row_loc, row_meas;
  std::vector<I4> rowrec;
  std::vector<double> br_g, br_bs, br_hb;
  std::vector<I4> slot;
  std::vector<I4> rslot;
  std::vector<I4> scon, rcon;  // contributions with their row record inline
  std::vector<int32_t> slot_rhs;  // per slot: 2 v for the diagonal slot of bus v, else -1
  std::vector<int32_t> cimg;      // per compact G block: its packed offset
  size_t lds = 0;
  for (int k = 0; k < K; ++k) {
    const AreaTemplates& t = p.tpl[k];
    AreaMeta a{};
    a.nn = p.sys[k].nn;
    a.nbr = (int32_t)t.br_lf.size();
    a.nrow = (int32_t)t.row_type.size();
    a.nslot = (c->area_lds && t.lds_split > 0) ? (int32_t)(t.cslot.size() + t.tslot.size())
                                                : (int32_t)t.slot.size();
    a.br = (int32_t)br_lf.size();
    br_lf.insert(br_lf.end(), t.br_lf.begin(), t.br_lf.end());
    br_lt.insert(br_lt.end(), t.br_lt.begin(), t.br_lt.end());
    br_g.insert(br_g.end(), t.br_g.begin(), t.br_g.end());
    br_bs.insert(br_bs.end(), t.br_bs.begin(), t.br_bs.end());
    br_hb.insert(br_hb.end(), t.br_hb.begin(), t.br_hb.end());
    a.inc_ptr = (int32_t)inc_ptr.size();
    append_rebased(inc_ptr, t.inc_ptr, (int32_t)inc_end.size());
    inc_end.insert(inc_end.end(), t.inc_end.begin(), t.inc_end.end());
    a.row = (int32_t)row_type.size();
    row_type.insert(row_type.end(), t.row_type.begin(), t.row_type.end());
    row_loc.insert(row_loc.end(), t.row_loc.begin(), t.row_loc.end());
    row_meas.insert(row_meas.end(), t.row_meas.begin(), t.row_meas.end());
    for (size_t r = 0; r < t.row_type.size(); ++r) rowrec.push_back({t.row_type[r], t.row_loc[r], t.row_meas[r], 0});
    // slots in order of decreasing contribution count, so that the lanes of
    // a wave carry similar loads (each slot writes its own storage).  For the
    // elimination in LDS the assembly writes the compact G blocks (offsets
    // relative to the area's value base) and the Schur-block slots of an area
    // that keeps that block in HBM; else every slot of the packed storage.
    a.slot = (int32_t)slot.size();
    a.gc_rel = p.gc_off[k] - p.val_off[k];
    a.n_cslot = 0;
    a.cimg = (int32_t)cimg.size();
    a.split = 0;
    {
      std::vector<I4> src;      // slot records with final offsets
      std::vector<int32_t> img; // packed offset of each
      if (c->area_lds && t.lds_split > 0) {
        for (size_t i = 0; i < t.cslot.size(); ++i) {
          const I4& q = t.cslot[i];
          src.push_back({q.x + a.gc_rel, q.y, q.z, q.w});
          img.push_back(t.cimg[i]);
          if (t.cimg[i] == p.sys[k].pin_off) sm[k].asm_pin = q.x + a.gc_rel;
        }
        for (const I4& q : t.tslot) {
          src.push_back(q);
          img.push_back(q.x);
        }
        a.n_cslot = (int32_t)t.cslot.size();
        a.split = t.lds_split;
        cimg.insert(cimg.end(), t.cimg.begin(), t.cimg.end());
      } else {
        for (const I4& q : t.slot) {
          src.push_back(q);
          img.push_back(q.x);
        }
      }
      std::vector<int> ord(src.size());
      for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        return src[x].w - src[x].z > src[y].w - src[y].z;
      });
      // a diagonal slot (v, v) also yields b_v: its contributions with equal
      // roles are exactly bus v's rhs contributions, in the same order
      std::unordered_map<int32_t, int32_t> diag_bus;
      for (int v = 0; v < p.sys[k].nn; ++v) diag_bus[p.sys[k].blk_off(v, v)] = v;
      // Contributions go to the device in P/Q pairs: the active and reactive
      // rows of one bus (injections) or one branch end (flows) have the same
      // support and roles, so one record evaluates both from one set of
      // branch terms.  Record {family | loc << 3, measurement of the P row or
      // -1, measurement of the Q row or -1, roles}; family VM, PINJ (for both
      // injections), PF or PT.
      std::map<std::pair<int, int>, int> row_of;  // (type, loc) -> row
      for (size_t r = 0; r < t.row_type.size(); ++r) row_of[{t.row_type[r], t.row_loc[r]}] = (int)r;
      auto partner = [&](int r) {
        const int ty = t.row_type[r];
        if (ty == MASE_VM) return -1;
        const bool isp = ty == MASE_PINJ || ty == MASE_PF || ty == MASE_PT;
        auto it = row_of.find({isp ? ty + 1 : ty - 1, t.row_loc[r]});
        return it == row_of.end() ? -1 : it->second;
      };
      // Pair records of every slot, then laid out for the kernel: slot i of
      // the area is handled by lane i % 64 of a wave, so the slots of each
      // run of 64 (one wave's, in this order) store their c-th records side
      // by side, at chunk base + c * 64 + lane; the chunk is as long as its
      // longest list (the slots are sorted by list length, so little is
      // padding).  Rows are the area's local rows.
      std::vector<std::vector<I4>> recs(ord.size());
      for (size_t n = 0; n < ord.size(); ++n) {
        const I4& q = src[ord[n]];
        std::map<std::pair<int, int>, bool> here;  // (row, roles) in this slot
        for (int c = q.z; c < q.w; ++c) here[{t.scon[c].x, t.scon[c].y}] = true;
        for (int c = q.z; c < q.w; ++c) {
          const int r = t.scon[c].x, roles = t.scon[c].y, ty = t.row_type[r];
          const int o = partner(r);
          const bool paired = o >= 0 && here.count({o, roles});
          const bool isq = ty == MASE_QINJ || ty == MASE_QF || ty == MASE_QT;
          if (paired && isq) continue;  // taken with its P row
          const int fam = ty == MASE_VM ? MASE_VM : (ty <= MASE_QINJ ? MASE_PINJ : (ty <= MASE_QF ? MASE_PF : MASE_PT));
          int32_t rp = -1, rq = -1;
          if (isq) rq = r;
          else { rp = r; if (paired) rq = o; }
          recs[n].push_back({fam | (t.row_loc[r] << 3), rp, rq, roles});
        }
      }
      for (size_t c0 = 0; c0 < ord.size(); c0 += 64) {
        const size_t c1 = std::min(ord.size(), c0 + 64);
        size_t len = 0;
        for (size_t n = c0; n < c1; ++n) len = std::max(len, recs[n].size());
        const int32_t base = (int32_t)scon.size();
        scon.resize(scon.size() + 64 * len, I4{0, -1, -1, 0});
        for (size_t n = c0; n < c1; ++n) {
          for (size_t c = 0; c < recs[n].size(); ++c) scon[base + c * 64 + (n - c0)] = recs[n][c];
          const I4& q = src[ord[n]];
          slot.push_back({q.x, q.y, base, (int32_t)recs[n].size()});
          slot_rhs.push_back(q.y < 0 ? 2 * diag_bus.at(img[ord[n]]) : -1);
        }
      }
    }
    // rhs items {cbeg, cend, bus}, by decreasing contribution count
    a.rslot = (int32_t)rslot.size();
    {
      std::vector<int> ord(t.rslot.size());
      for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        return t.rslot[x].y - t.rslot[x].x > t.rslot[y].y - t.rslot[y].x;
      });
      for (int v : ord)
        rslot.push_back({t.rslot[v].x + (int32_t)rcon.size(), t.rslot[v].y + (int32_t)rcon.size(), v, 0});
    }
    for (const I2& cc : t.rcon)
      rcon.push_back({t.row_type[cc.x], t.row_loc[cc.x], t.row_meas[cc.x], cc.y});
    a.tail_src = p.tail_src_ptr[k];
    a.slack_local = p.local_of_bus[k][p.slack];
    am[k] = a;
  }
  int dev = 0, maxlds = 0, n_cu = 0;
  HIPTRY(hipGetDevice(&dev));
  HIPTRY(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  HIPTRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  // stage branch records in LDS when every area fits
  // (and the rows' weights and measurements, when they fit as well)
  size_t lds_br = 0, lds_nobr = 0, lds_br_wz = 0, lds_nobr_wz = 0;
  for (int k = 0; k < K; ++k) {
    lds_br = std::max(lds_br, assemble_lds_bytes(am[k].nn, am[k].nbr, true, 0));
    lds_nobr = std::max(lds_nobr, assemble_lds_bytes(am[k].nn, am[k].nbr, false, 0));
    lds_br_wz = std::max(lds_br_wz, assemble_lds_bytes(am[k].nn, am[k].nbr, true, am[k].nrow));
    lds_nobr_wz = std::max(lds_nobr_wz, assemble_lds_bytes(am[k].nn, am[k].nbr, false, am[k].nrow));
  }
  c->d.asm_wz = 0;
  if (lds_br_wz <= (size_t)maxlds) {
    c->br_lds = true;
    c->d.asm_wz = 1;
    lds = lds_br_wz;
  } else if (lds_nobr_wz <= (size_t)maxlds) {
    c->br_lds = false;
    c->d.asm_wz = 1;
    lds = lds_nobr_wz;
  } else {
    c->br_lds = lds_br <= (size_t)maxlds;
    lds = c->br_lds ? lds_br : lds_nobr;
  }
  // an area too large to stage in LDS: every area stages in its own region
  // of HBM instead (same arithmetic)
  int64_t asm_stride = 0;
  if (lds > (size_t)maxlds) {
    for (int k = 0; k < K; ++k) {
      am[k].stage_off = (int32_t)asm_stride;
      asm_stride += ((8 * (int64_t)am[k].nn + 2 * (int64_t)am[k].nbr) + 31) / 32 * 32;
    }
    c->br_lds = false;
    c->d.asm_wz = 0;
    lds = 0;
  }
  c->lds_asm = lds;
  c->lds_el_area = 0;
  for (int k = 0; k < K; ++k) c->lds_el_area = std::max(c->lds_el_area, 8 * (size_t)p.sys[k].lds_doubles);
  c->lds_el_gamma = 8 * (size_t)p.sys[K].lds_doubles;
  if (std::max(c->lds_el_area, c->lds_el_gamma) > 65536)
    HIPTRY(allow_eliminate_lds(std::max(c->lds_el_area, c->lds_el_gamma)));
  // boundary dense block: the widest panel (up to 64 columns) that fits in
  // LDS, else 16-column panels in LDS, else the matrix in HBM only
  // (MASE_DENSE_PANEL=0/1/2 forces one of these)
  {
    const int ld = p.sys[K].ld;
    const char* env = getenv("MASE_DENSE_PANEL");
    int nb = 64;
    while (nb >= 16 && dense_lds_bytes(ld, DENSE_WIDE, nb) + 8192 > (size_t)maxlds) nb -= 16;
    c->dense_nb = nb;
    if (nb >= 16) c->dense_mode = DENSE_WIDE;
    else if (dense_lds_bytes(ld, DENSE_PANEL16, 16) + 8192 <= (size_t)maxlds) c->dense_mode = DENSE_PANEL16;
    else c->dense_mode = DENSE_GLOBAL;
    if (env && env[0] >= '0' && env[0] <= '2' && env[0] - '0' <= c->dense_mode) c->dense_mode = env[0] - '0';
    if (c->dense_mode == DENSE_WIDE) c->dense_nb = std::max(16, c->dense_nb);
    const size_t bytes = dense_lds_bytes(ld, c->dense_mode, c->dense_nb);
    if (c->dense_mode != DENSE_GLOBAL && bytes > 65536) HIPTRY(allow_dense_lds(c->dense_mode, bytes));
    // the autotuner may also pick 16-column panels in LDS
    const size_t b16 = dense_lds_bytes(ld, DENSE_PANEL16, 16);
    if (c->dense_mode == DENSE_WIDE && b16 > 65536) HIPTRY(allow_dense_lds(DENSE_PANEL16, b16));
  }
  // supernodal boundary elimination (MASE_GAMMA_SNODE=0 selects the level engine)
  {
    const char* env = getenv("MASE_GAMMA_SNODE");
    c->lds_sn = (size_t)p.sys[K].sn_lds_bytes;
    c->snode_possible = !p.sys[K].sn.empty() && c->lds_sn + 8192 <= (size_t)maxlds;
    c->gamma_snode = c->snode_possible && !(env && env[0] == '0');
    if (c->snode_possible && c->lds_sn > 65536) {
      HIPTRY(allow_gamma_snode_lds(c->lds_sn));
      HIPTRY(allow_gamma_snode_back_lds(c->lds_sn));
    }
    // subtree groups: as many workgroups per snapshot as fit the device at
    // once for the whole batch (MASE_SNODE_GROUPS overrides the limit)
    const int per_cu = std::max(1, (int)(160 * 1024 / std::max<size_t>(c->lds_sn, 1)));
    int gmax = std::max(1, n_cu * per_cu / std::max(1, p.n_snap));
    const char* genv = getenv("MASE_SNODE_GROUPS");
    if (genv && atoi(genv) > 0) gmax = atoi(genv);
    c->plan.sys[K].group_supernodes(gmax);
  }
  c->hsys = sm;
  c->nslot_g = (int)p.g_slot.size();

  Dev& d = c->d;
  d.n_bus = p.n_bus; d.n_meas = p.n_meas; d.n_area = K; d.n_snap = p.n_snap; d.slack = p.slack;
  d.bs_max_nn_area = 0;
  for (int k = 0; k < K; ++k) d.bs_max_nn_area = std::max(d.bs_max_nn_area, (int32_t)p.sys[k].nn);
  d.bs_max_nn_gamma = p.sys[K].nn;
  d.vstride = p.vstride; d.rstride = p.rstride;
  int rc = 0;
#define UP(field, vec) if ((rc = upload(c, vec, &d.field))) return rc
  if (c->area_lds) {
    // launch order: largest LDS need first; consecutive areas with the same
    // workgroups per CU share a launch (the LDS size is per launch)
    // areas that do not fit (split 0) come first and run the level engine
    std::vector<int32_t>& ord = c->plan.area_order;
    auto need = [&](int k) {
      return am[k].split > 0 ? 8 * ((size_t)am[k].split + 2 * (size_t)p.sys[k].nn) : SIZE_MAX;
    };
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return need(x) > need(y); });
    const size_t per_cu = 8 * (size_t)AREA_LDS_DOUBLES;
    const char* ntenv = getenv("MASE_ELIM_NT");
    const int nt_force = ntenv ? atoi(ntenv) : 0;
    size_t lds_max = 0;
    int q = 0;
    while (q < K && am[ord[q]].split == 0) ++q;
    if (q > 0) c->el_class.push_back({0, q, 0, 0, false, 0});
    while (q < K) {
      const int k0 = ord[q];
      const size_t b0 = need(k0);
      const int wpc = (int)std::min<size_t>(8, std::max<size_t>(1, per_cu / b0));
      int r = q;
      bool tail = false;
      while (r < K && (int)std::min<size_t>(8, std::max<size_t>(1, per_cu / need(ord[r]))) == wpc) {
        tail |= am[ord[r]].split < p.sys[ord[r]].nval;
        ++r;
      }
      const int nt = (nt_force == 256 || nt_force == 512 || nt_force == 1024) ? nt_force
                     : wpc == 1 ? 1024 : (wpc <= 4 ? 512 : 256);
      c->el_class.push_back({q, r - q, b0, nt, tail, nt});
      lds_max = std::max(lds_max, b0);
      q = r;
    }

    if (lds_max > (size_t)maxlds) {
      c->el_class.clear();
      c->area_lds = false;
      return fail(MASE_ERR_ARG, "an area's elimination needs more LDS than the device allows");
    }
    if (lds_max > 65536) HIPTRY(allow_elim_lds(lds_max));
  }
  UP(sys, sm); UP(area, am); UP(area_order, p.area_order); UP(gbus, gbus);
  UP(br_lf, br_lf); UP(br_lt, br_lt); UP(br_g, br_g); UP(br_bs, br_bs); UP(br_hb, br_hb);
  UP(inc_ptr, inc_ptr); UP(inc_end, inc_end);
  UP(row_type, row_type); UP(row_loc, row_loc); UP(row_meas, row_meas); UP(rowrec, rowrec);
  UP(slot, slot); UP(scon, scon); UP(rslot, rslot); UP(rcon, rcon); UP(slot_rhs, slot_rhs);
  UP(cd_ptr, cd_ptr); UP(up_ptr, up_ptr); UP(rb_ptr, rb_ptr); UP(bs_ptr, bs_ptr); UP(bs_lg, bs_lg);
  UP(cd_items, cd_items); UP(up_tgt, up_tgt); UP(up_con, up_con);
  UP(rb_tgt, rb_tgt); UP(rb_con, rb_con); UP(bs_items, bs_items); UP(bs_con, bs_con);
  UP(up_tgt_img, up_tgt_img); UP(up_con_img, up_con_img); UP(rb_con_img, rb_con_img); UP(cimg, cimg);
  {
    const SysPlan& gs = p.sys[K];
    d.n_sn = (int32_t)gs.sn.size();
    UP(sn, gs.sn); UP(sn2, gs.sn2); UP(sn_rows, gs.sn_rows); UP(sn_tgt, gs.sn_tgt);
    d.n_sn_grp = (int32_t)gs.sn_grp_ptr.size() - 1;
    UP(sn_grp_ptr, gs.sn_grp_ptr); UP(sn_grp, gs.sn_grp);
    UP(sn3, gs.sn3); UP(tail_ent, gs.tail_ent); UP(tail_con, gs.tail_con);
    d.n_tail_ent = (int32_t)gs.tail_ent.size();
    d.tl_stride = gs.tl_doubles;
    d.sn_tl = nullptr;
    if (gs.tl_doubles > 0 && (rc = dalloc(c, (size_t)gs.tl_doubles * p.n_snap, &d.sn_tl))) return rc;
  }
  UP(g_slot, p.g_slot); UP(g_con, p.g_con); UP(g_rslot, p.g_rslot); UP(g_rcon, p.g_rcon);
  UP(tail_src, p.tail_src); UP(bus_dx_src, p.bus_dx_src);
#undef UP
  const int64_t S = p.n_snap;
  double* z = nullptr;
  double* w = nullptr;
  if ((rc = dalloc(c, S * p.n_meas, &z))) return rc;
  if ((rc = dalloc(c, p.n_meas, &w))) return rc;
  d.z = z;
  d.w = w;
  std::vector<double> w0(p.n_meas);
  for (int i = 0; i < p.n_meas; ++i) w0[i] = 1.0 / (p.sigma[i] * p.sigma[i]);
  HIPTRY(hipMemcpy(w, w0.data(), sizeof(double) * p.n_meas, hipMemcpyHostToDevice));
  if ((rc = dalloc(c, p.n_meas, &c->w_default))) return rc;
  d.asm_stage = nullptr;
  d.asm_stride = asm_stride;
  if (asm_stride > 0 && (rc = dalloc(c, (size_t)(asm_stride * S), &d.asm_stage))) return rc;
  HIPTRY(hipMemcpy(c->w_default, w0.data(), sizeof(double) * p.n_meas, hipMemcpyHostToDevice));
  if ((rc = dalloc(c, S * p.n_bus, &d.x))) return rc;
  if ((rc = dalloc(c, S * p.n_bus, &c->xscratch))) return rc;
  if ((rc = dalloc(c, S * p.n_bus, &c->stage_vm))) return rc;
  if ((rc = dalloc(c, S * p.n_bus, &c->stage_va))) return rc;
  if ((rc = dalloc(c, S * p.vstride, &d.vals))) return rc;
  if ((rc = dalloc(c, S * p.rstride, &d.rhs))) return rc;
  if ((rc = dalloc(c, S * K, &d.jpart))) return rc;
  // per-snapshot flags in one block, {maxdx [S] | active [S] | status [S][K+1] | iters [S]},
  // so that one copy brings an iteration's outcome to the host
  const size_t flag_bytes = sizeof(double) * S + sizeof(int32_t) * (S * (K + 2) + S);
  {
    double* blk = nullptr;
    if ((rc = dalloc(c, (flag_bytes + 7) / 8, &blk))) return rc;
    d.maxdx = blk;
    d.active = reinterpret_cast<int32_t*>(blk + S);
    d.status = d.active + S;
    d.iters = d.status + S * (K + 1);
  }
  if ((rc = dalloc(c, 1, &c->dtol))) return rc;
  d.tol = c->dtol;
  d.hout = nullptr;
  HIPTRY(hipMemset(d.vals, 0, sizeof(double) * S * p.vstride));
  HIPTRY(hipMemset(d.rhs, 0, sizeof(double) * S * p.rstride));
  HIPTRY(hipHostMalloc((void**)&c->h_maxdx, (flag_bytes + 7) / 8 * 8, hipHostMallocDefault));
  c->h_active = reinterpret_cast<int32_t*>(c->h_maxdx + S);
  c->h_status = c->h_active + S;
  c->h_iters = c->h_status + S * (K + 1);
  HIPTRY(hipHostMalloc((void**)&c->h_tol, sizeof(double), hipHostMallocDefault));
  c->h_tol[0] = 1e-6;
  // stream solve: active flags and stream positions of two alternate passes
  HIPTRY(hipHostMalloc((void**)&c->h_st_active, sizeof(int32_t) * (2 * (size_t)S + 4), hipHostMallocDefault));
  c->h_st_pos = c->h_st_active + 2 * S;
  // the refill kernel writes them directly (no copy per pass)
  HIPTRY(hipHostGetDevicePointer((void**)&c->h_st_active_dev, c->h_st_active, 0));
  c->h_st_pos_dev = c->h_st_active_dev + 2 * S;
  for (auto& e : c->st_ev) HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPTRY(hipMemcpy(c->dtol, c->h_tol, sizeof(double), hipMemcpyHostToDevice));

  if (c->lds_asm > (size_t)maxlds)
    return fail(MASE_ERR_ARG, "an area needs " + std::to_string(c->lds_asm) +
                                  " bytes of LDS for assembly; the device allows " +
                                  std::to_string(maxlds));
  if (c->lds_asm > 65536) HIPTRY(allow_assemble_lds(c->lds_asm, c->br_lds));
  return 0;
}

const SysMeta& gsys(const mase_ctx* c) { return c->hsys[c->plan.n_area]; }

struct StageMark {
  mase_ctx* c;
  hipStream_t st;
  int stage;
  StageMark(mase_ctx* c_, hipStream_t st_, int s_) : c(c_), st(st_), stage(s_) {
    if (c->prof) {
      (void)hipEventRecord(c->pev[2 * stage], st);
      c->pused[stage] = true;
    }
  }
  ~StageMark() {
    if (c->prof) (void)hipEventRecord(c->pev[2 * stage + 1], st);
  }
};

bool snapshot_bad(const mase_ctx* c, int s);

// The areas' elimination (stage 2) for the areas at positions [a0, a0 + na)
// of area_order and snapshots [s0, s0 + ns): held in LDS class by class, or
// the level engine over HBM.
hipError_t launch_area_eliminate(const mase_ctx* c, int a0, int na, int s0, int ns, hipStream_t st) {
  if (!c->area_lds) return launch_eliminate(c->d, a0, na, s0, ns, c->lds_el_area, st);
  for (const auto& cl : c->el_class) {
    const int lo = std::max(a0, cl.a0), hi = std::min(a0 + na, cl.a0 + cl.na);
    if (lo >= hi) continue;
    // nt 0: areas too large for LDS, on the level engine
    const hipError_t e = cl.nt ? launch_elim_lds(c->d, lo, hi - lo, s0, ns, cl.lds, cl.nt, cl.tail_hbm, st)
                               : launch_eliminate(c->d, lo, hi - lo, s0, ns, c->lds_el_area, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The areas' back substitution (stage 4a) for the same positions: the factor
// read into LDS for the areas eliminated there (the class's LDS size covers
// the factor and the rhs), else the level engine over HBM.
hipError_t launch_area_backsolve(const mase_ctx* c, int a0, int na, int s0, int ns, hipStream_t st,
                                 bool fixed_bnd = false) {
  if (!c->area_lds) return launch_backsolve(c->d, a0, na, s0, ns, st, fixed_bnd);
  for (const auto& cl : c->el_class) {
    const int lo = std::max(a0, cl.a0), hi = std::min(a0 + na, cl.a0 + cl.na);
    if (lo >= hi) continue;
    const hipError_t e = cl.nt ? launch_back_lds(c->d, lo, hi - lo, s0, ns, cl.lds, cl.nt, fixed_bnd, st)
                               : launch_backsolve(c->d, lo, hi - lo, s0, ns, st, fixed_bnd);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Stages 1-2 (assembly, condensation) for snapshots [s0, s0 + ns), after
// the iteration's local steps (Eq. 6: each area's internal variables take
// GN steps with its boundary held; same kernels, dx_b = 0).
int launch_area_part(mase_ctx* c, hipStream_t st, int s0, int ns) {
  const int K = c->plan.n_area;
  const Dev& d = c->d;
  if (c->opt.local_steps > 0) {
    StageMark m(c, st, MASE_STAGE_LOCAL);
    for (int l = 0; l < c->opt.local_steps; ++l) {
      HIPTRY(launch_assemble(d, 0, K, s0, ns, MODE_ASSEMBLE, c->lds_asm, c->br_lds, st));
      HIPTRY(launch_area_eliminate(c, 0, K, s0, ns, st));
      HIPTRY(launch_area_backsolve(c, 0, K, s0, ns, st, true));
      HIPTRY(launch_update(d, s0, ns, st, true));
    }
  }
  {
    StageMark m(c, st, MASE_STAGE_ASSEMBLE);
    HIPTRY(launch_assemble(d, 0, K, s0, ns, MODE_ASSEMBLE, c->lds_asm, c->br_lds, st));
  }
  {
    StageMark m(c, st, MASE_STAGE_CONDENSE);
    HIPTRY(launch_area_eliminate(c, 0, K, s0, ns, st));
  }
  return 0;
}

// Stages 3-4 (boundary assembly and solve, back substitution, update) for
// snapshots [s0, s0 + ns).
int launch_gamma_part(mase_ctx* c, hipStream_t st, int s0, int ns) {
  const int K = c->plan.n_area;
  const Dev& d = c->d;
  const SysMeta& g = gsys(c);
  if (g.nn > 0) {
    {
      StageMark m(c, st, MASE_STAGE_GAMMA_GATHER);
      HIPTRY(launch_gamma_gather(d, s0, ns, c->nslot_g, g.nn, st));
    }
    if (g.ne > 0) {
      StageMark m(c, st, MASE_STAGE_GAMMA_SPARSE);
      HIPTRY(launch_gamma_sparse(c, s0, ns, st));
    }
    {
      StageMark m(c, st, MASE_STAGE_GAMMA_DENSE);
      HIPTRY(launch_dense_chol(d, s0, ns, g.ld, c->dense_mode, c->dense_nb, st));
    }
    if (g.ne > 0) {
      StageMark m(c, st, MASE_STAGE_GAMMA_BACK);
      HIPTRY(launch_gamma_back(c, s0, ns, st));
    }
  }
  {
    StageMark m(c, st, MASE_STAGE_BACKSOLVE);
    HIPTRY(launch_area_backsolve(c, 0, K, s0, ns, st));
  }
  {
    StageMark m(c, st, MASE_STAGE_UPDATE);
    HIPTRY(launch_update(d, s0, ns, st));
  }
  return 0;
}

int launch_batched_iteration(mase_ctx* c, hipStream_t st) {
  const int S = c->plan.n_snap;
  for (bool& u : c->pused) u = false;
  int rc = launch_area_part(c, st, 0, S);
  if (rc) return rc;
  return launch_gamma_part(c, st, 0, S);
}

// Captures fn(c, st, s0, ns) on stream st as an executable graph.
int capture_part(mase_ctx* c, hipStream_t st, int (*fn)(mase_ctx*, hipStream_t, int, int), int s0, int ns,
                 hipGraphExec_t* out) {
  HIPTRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int rc = fn(c, st, s0, ns);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return fail(MASE_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  c->pgraphs.push_back(g);
  HIPTRY(hipGraphInstantiate(out, g, nullptr, nullptr, 0));
  return 0;
}

// Streams, events and the two graphs per group of the pipelined solve.
int setup_pipeline(mase_ctx* c) {
  if (!c->pgA.empty()) return 0;
  const int G = c->npipe, S = c->plan.n_snap;
  c->pg_s0.resize(G + 1);
  for (int g = 0; g <= G; ++g) c->pg_s0[g] = (int)((int64_t)S * g / G);
  HIPTRY(hipStreamCreateWithFlags(&c->pstream_area, hipStreamNonBlocking));
  c->pstream.assign(G, nullptr);
  c->pev_a.assign(G, nullptr);
  c->pev_b.assign(G, nullptr);
  c->pgA.assign(G, nullptr);
  c->pgB.assign(G, nullptr);
  for (int g = 0; g < G; ++g) {
    HIPTRY(hipStreamCreateWithFlags(&c->pstream[g], hipStreamNonBlocking));
    HIPTRY(hipEventCreateWithFlags(&c->pev_a[g], hipEventDisableTiming));
    HIPTRY(hipEventCreateWithFlags(&c->pev_b[g], hipEventDisableTiming));
  }
  for (int g = 0; g < G; ++g) {
    const int s0 = c->pg_s0[g], ns = c->pg_s0[g + 1] - s0;
    int rc = capture_part(c, c->pstream_area, launch_area_part, s0, ns, &c->pgA[g]);
    if (rc) return rc;
    rc = capture_part(c, c->pstream[g], launch_gamma_part, s0, ns, &c->pgB[g]);
    if (rc) return rc;
  }
  return 0;
}

// One iteration of group g: area stages on the shared area stream, then the
// boundary solve and update on the group's stream, then its flags to host.
int launch_group_iteration(mase_ctx* c, int g) {
  const int K = c->plan.n_area;
  const int s0 = c->pg_s0[g], ns = c->pg_s0[g + 1] - s0;
  HIPTRY(hipStreamWaitEvent(c->pstream_area, c->pev_b[g], 0));
  HIPTRY(hipGraphLaunch(c->pgA[g], c->pstream_area));
  HIPTRY(hipEventRecord(c->pev_a[g], c->pstream_area));
  hipStream_t st = c->pstream[g];
  HIPTRY(hipStreamWaitEvent(st, c->pev_a[g], 0));
  HIPTRY(hipGraphLaunch(c->pgB[g], st));
  HIPTRY(hipMemcpyAsync(c->h_active + s0, c->d.active + s0, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
  HIPTRY(hipMemcpyAsync(c->h_maxdx + s0, c->d.maxdx + s0, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
  HIPTRY(hipMemcpyAsync(c->h_status + (size_t)s0 * (K + 1), c->d.status + (size_t)s0 * (K + 1),
                        sizeof(int32_t) * ns * (K + 1), hipMemcpyDeviceToHost, st));
  HIPTRY(hipEventRecord(c->pev_b[g], st));
  return 0;
}

// mase_solve's batched graph schedule with snapshot groups that iterate
// independently: the host waits for the groups round-robin and relaunches
// each one that still has active snapshots, so a group's boundary solve runs
// while the next group's area stages occupy the chip.  Each snapshot goes
// through exactly the kernels and arithmetic of the one-group schedule.
int pipelined_solve(mase_ctx* c, int max_iter) {
  int rc = setup_pipeline(c);
  if (rc) return rc;
  const int G = c->npipe;
  HIPTRY(hipEventRecord(c->ev_main, c->stream));
  HIPTRY(hipStreamWaitEvent(c->pstream_area, c->ev_main, 0));
  for (int g = 0; g < G; ++g) {
    HIPTRY(hipStreamWaitEvent(c->pstream[g], c->ev_main, 0));
    HIPTRY(hipEventRecord(c->pev_b[g], c->pstream[g]));
  }
  std::vector<int> done(G, 0), iters(G, 0);
  auto group_active = [&](int g) {
    for (int s = c->pg_s0[g]; s < c->pg_s0[g + 1]; ++s)
      if (c->h_active[s]) return true;
    return false;
  };
  int pending = 0;
  for (int g = 0; g < G; ++g) {
    if (!group_active(g)) { done[g] = 1; continue; }
    if ((rc = launch_group_iteration(c, g))) return rc;
    ++pending;
  }
  while (pending > 0) {
    for (int g = 0; g < G; ++g) {
      if (done[g]) continue;
      HIPTRY(hipEventSynchronize(c->pev_b[g]));
      ++iters[g];
      // a snapshot with a non-positive pivot is frozen (inactive) by the
      // update kernel, so its group goes on with the others
      if (!group_active(g) || iters[g] >= max_iter) {
        done[g] = 1;
        --pending;
        continue;
      }
      if ((rc = launch_group_iteration(c, g))) return rc;
    }
  }
  // later work on the context's stream follows every group
  HIPTRY(hipEventRecord(c->ev_main, c->pstream_area));
  HIPTRY(hipStreamWaitEvent(c->stream, c->ev_main, 0));
  for (int g = 0; g < G; ++g) HIPTRY(hipStreamWaitEvent(c->stream, c->pev_b[g], 0));
  return 0;
}

// After a synchronised iteration: add each recorded stage's elapsed time.
int accumulate_profile(mase_ctx* c, int nactive) {
  if (!c->prof) return 0;
  for (int i = 0; i < MASE_N_STAGE; ++i) {
    if (!c->pused[i]) continue;
    float ms = 0.f;
    HIPTRY(hipEventElapsedTime(&ms, c->pev[2 * i], c->pev[2 * i + 1]));
    c->pms[i] += ms;
    c->plaunch[i] += 1;
    c->punits[i] += nactive;
  }
  return 0;
}

// The paper's schedule for one snapshot: per-area launches on per-area
// streams for assembly + condensation, boundary work on the main stream,
// per-area back substitution on the area streams again (Section 4.3).
int launch_plain_iteration(mase_ctx* c, int s) {
  const int K = c->plan.n_area;
  const Dev& d = c->d;
  hipStream_t st = c->stream;
  const int ns = (int)c->astreams.size();
  HIPTRY(hipEventRecord(c->ev_main, st));
  for (int i = 0; i < ns; ++i) HIPTRY(hipStreamWaitEvent(c->astreams[i], c->ev_main, 0));
  for (int ai = 0; ai < K; ++ai) {
    hipStream_t as = c->astreams[ai % ns];
    HIPTRY(launch_assemble(d, ai, 1, s, 1, MODE_ASSEMBLE, c->lds_asm, c->br_lds, as));
    HIPTRY(launch_area_eliminate(c, ai, 1, s, 1, as));
  }
  for (int i = 0; i < ns; ++i) {
    HIPTRY(hipEventRecord(c->aevents[i], c->astreams[i]));
    HIPTRY(hipStreamWaitEvent(st, c->aevents[i], 0));
  }
  const SysMeta& g = gsys(c);
  if (g.nn > 0) {
    HIPTRY(launch_gamma_gather(d, s, 1, c->nslot_g, g.nn, st));
    if (g.ne > 0) HIPTRY(launch_gamma_sparse(c, s, 1, st));
    HIPTRY(launch_dense_chol(d, s, 1, g.ld, c->dense_mode, c->dense_nb, st));
    if (g.ne > 0) HIPTRY(launch_gamma_back(c, s, 1, st));
  }
  HIPTRY(hipEventRecord(c->ev_main, st));
  for (int i = 0; i < ns; ++i) HIPTRY(hipStreamWaitEvent(c->astreams[i], c->ev_main, 0));
  for (int ai = 0; ai < K; ++ai) HIPTRY(launch_area_backsolve(c, ai, 1, s, 1, c->astreams[ai % ns]));
  for (int i = 0; i < ns; ++i) {
    HIPTRY(hipEventRecord(c->aevents[i], c->astreams[i]));
    HIPTRY(hipStreamWaitEvent(st, c->aevents[i], 0));
  }
  HIPTRY(launch_update(d, s, 1, st));
  return 0;
}

int read_flags(mase_ctx* c) {
  const int S = c->plan.n_snap, K = c->plan.n_area;
  // maxdx, active and status are contiguous on both sides
  HIPTRY(hipMemcpyAsync(c->h_maxdx, c->d.maxdx, sizeof(double) * S + sizeof(int32_t) * S * (K + 2),
                        hipMemcpyDeviceToHost, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  return 0;
}

bool snapshot_bad(const mase_ctx* c, int s) {
  const int K = c->plan.n_area;
  for (int k = 0; k <= K; ++k)
    if (c->h_status[(size_t)s * (K + 1) + k]) return true;
  return false;
}

int check_device(const mase_ctx* c) {
  if (!c) return fail(MASE_ERR_ARG, "null context");
  if (c->host_only) return fail(MASE_ERR_NO_DEVICE, "context was created host-only");
  return 0;
}

// Canonical index of (local bus v, component comp) of system k, or -1 for
// the slack angle.  For areas the canonical order is internal buses
// ascending then boundary buses ascending; for the boundary system it is
// Gamma order.
std::vector<int32_t> canon_index(const Plan& p, int k) {
  const SysPlan& s = p.sys[k];
  std::vector<int32_t> out(2 * s.nn, -1);
  std::vector<std::pair<int, int>> key;  // (rank, local)
  for (int v = 0; v < s.nn; ++v) {
    int rank;
    if (k < p.n_area) rank = (v < s.ne ? 0 : 1) * p.n_bus + s.gbus[v];
    else rank = p.gamma_canon_pos[s.gbus[v]];
    key.push_back({rank, v});
  }
  std::sort(key.begin(), key.end());
  int c = 0;
  for (auto& kv : key) {
    const int v = kv.second;
    if (s.gbus[v] != p.slack) out[2 * v] = c++;
    out[2 * v + 1] = c++;
  }
  return out;
}

// Dense symmetric matrix (row-major, dim x dim) of system k's packed blocks
// whose row and column both satisfy `take`, in canonical order offset by off.
template <class F>
void unpack_blocks(const Plan& p, int k, const std::vector<double>& vals, const std::vector<int32_t>& ci,
                   int dim, int off, F take, double* M) {
  const SysPlan& s = p.sys[k];
  auto put = [&](int i, int j, int32_t o, int32_t stride) {
    for (int r = 0; r < 2; ++r)
      for (int cc = 0; cc < 2; ++cc) {
        const int a = ci[2 * i + r], b = ci[2 * j + cc];
        if (a < 0 || b < 0 || !take(i) || !take(j)) continue;
        const double v = vals[o + r + cc * stride];
        M[(size_t)(a - off) * dim + (b - off)] = v;
        M[(size_t)(b - off) * dim + (a - off)] = v;
      }
  };
  for (int j = 0; j < s.ne; ++j) {
    put(j, j, s.col_off[j], 2);
    for (int i : s.strct[j]) put(i, j, s.blk_off(i, j), 2);
  }
  for (int q = s.ne; q < s.nn; ++q)
    for (int i = q; i < s.nn; ++i) put(i, q, s.blk_off(i, q), s.blk_stride(i, q));
}

}  // namespace

namespace mase {

int set_error(int code, const std::string& msg) { return fail(code, msg); }

int objective_at(mase_ctx* c, double2* x, double* jpart) {
  Dev d = c->d;
  d.x = x;
  d.jpart = jpart;
  HIPTRY(launch_assemble(d, 0, c->plan.n_area, 0, c->plan.n_snap, MODE_OBJECTIVE, c->lds_asm, c->br_lds,
                         c->stream));
  return 0;
}

}  // namespace mase

extern "C" {

void mase_default_options(mase_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->batched = 1;
  opt->use_graph = 1;
  opt->gamma_mode = MASE_GAMMA_SPARSE;
}

const char* mase_last_error(void) { return g_err.c_str(); }

const char* mase_strerror(int code) {
  switch (code) {
    case MASE_OK: return "ok";
    case MASE_NOT_CONVERGED: return "not converged";
    case MASE_ERR_ARG: return "invalid argument";
    case MASE_ERR_STATE: return "call out of order";
    case MASE_ERR_NOT_POSDEF: return "non-positive pivot (unobservable system)";
    case MASE_ERR_HIP: return "HIP runtime error";
    case MASE_ERR_OOM: return "out of memory";
    case MASE_ERR_NO_DEVICE: return "host-only context";
    default: return "unknown error";
  }
}

int mase_create(int32_t n_bus, int32_t n_branch, const int32_t* br_from, const int32_t* br_to,
                const double* br_r, const double* br_x, const double* br_b, int32_t slack_bus,
                int32_t n_area, const int32_t* bus_area, int32_t n_meas, const int32_t* meas_type,
                const int32_t* meas_at, const double* meas_sigma, int32_t n_snap,
                const mase_options* opt, mase_ctx** out) {
  if (!out) return fail(MASE_ERR_ARG, "out is null");
  *out = nullptr;
  mase_options o;
  mase_default_options(&o);
  if (opt) o = *opt;
  Input in{n_bus, n_branch, br_from, br_to, br_r, br_x, br_b, slack_bus, n_area, bus_area,
           n_meas, meas_type, meas_at, meas_sigma, n_snap, o.gamma_mode};
  if (o.pipeline_groups < 0) return fail(MASE_ERR_ARG, "pipeline_groups must be >= 0");
  if (o.local_steps < 0) return fail(MASE_ERR_ARG, "local_steps must be >= 0");
  if (o.local_steps > 0 && !o.batched) return fail(MASE_ERR_ARG, "local_steps needs the batched schedule");
  mase_ctx* c = new (std::nothrow) mase_ctx();
  if (!c) return fail(MASE_ERR_OOM, "host allocation failed");
  c->opt = o;
  c->npipe = o.pipeline_groups > 0 ? o.pipeline_groups : 1;
  c->npipe = std::max(1, std::min(c->npipe, std::max(1, n_snap)));
  if (o.tune_cache) c->tune_path = o.tune_cache;
  c->opt.tune_cache = nullptr;  // the caller's string is not kept
  c->host_only = o.host_only != 0;
  std::string err;
  try {
    err = build_plan(in, c->plan);
  } catch (std::exception& ex) {
    err = std::string("setup failed: ") + ex.what();
  }
  if (!err.empty()) {
    delete c;
    return fail(MASE_ERR_ARG, err);
  }
  if (c->host_only) {
    *out = c;
    return 0;
  }
  int rc = 0;
  if (o.stream) {
    c->stream = (hipStream_t)o.stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) { delete c; return fail(MASE_ERR_HIP, hipGetErrorString(e)); }
    c->own_stream = true;
  }
  if (!o.batched) {
    const int ns = std::max(1, std::min(n_area, 32));
    c->astreams.resize(ns);
    c->aevents.resize(ns);
    for (int i = 0; i < ns && !rc; ++i) {
      if (hipStreamCreateWithFlags(&c->astreams[i], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&c->aevents[i], hipEventDisableTiming) != hipSuccess)
        rc = fail(MASE_ERR_HIP, "stream creation failed");
    }
  }
  if (!rc && hipEventCreateWithFlags(&c->ev_main, hipEventDisableTiming) != hipSuccess)
    rc = fail(MASE_ERR_HIP, "event creation failed");
  if (!rc) rc = upload_plan(c);
  if (!rc) rc = scratch_address(&c->noalloc_scratch);
  if (!rc) {
    hipError_t e = launch_pack_state(c->d, nullptr, nullptr, c->d.x, c->stream);
    if (e == hipSuccess) e = launch_reset_flags(c->d, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail(MASE_ERR_HIP, hipGetErrorString(e));
  }
  if (rc) {
    mase_destroy(c);
    return rc;
  }
  *out = c;
  return 0;
}

void mase_destroy(mase_ctx* c) {
  if (!c) return;
  if (!c->host_only) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->pstream_area) (void)hipStreamSynchronize(c->pstream_area);
    for (auto s : c->pstream) if (s) (void)hipStreamSynchronize(s);
    for (auto e : c->pgA) if (e) (void)hipGraphExecDestroy(e);
    for (auto e : c->pgB) if (e) (void)hipGraphExecDestroy(e);
    for (auto g : c->pgraphs) if (g) (void)hipGraphDestroy(g);
    for (auto e : c->pev_a) if (e) (void)hipEventDestroy(e);
    for (auto e : c->pev_b) if (e) (void)hipEventDestroy(e);
    for (auto s : c->pstream) if (s) (void)hipStreamDestroy(s);
    if (c->pstream_area) (void)hipStreamDestroy(c->pstream_area);
    for (auto s : c->astreams) if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
    for (auto e : c->aevents) if (e) (void)hipEventDestroy(e);
    if (c->ev_main) (void)hipEventDestroy(c->ev_main);
    for (auto e : c->pev) if (e) (void)hipEventDestroy(e);
    for (void* p : c->dallocs) (void)hipFree(p);
    if (c->h_maxdx) (void)hipHostFree(c->h_maxdx);  // also holds h_active, h_status, h_iters
    if (c->h_tol) (void)hipHostFree(c->h_tol);
    if (c->st_out) (void)hipFree(c->st_out);
    if (c->h_st_active) (void)hipHostFree(c->h_st_active);
    for (auto e : c->st_ev) if (e) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

int mase_set_measurements(mase_ctx* c, const double* z, const double* w) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!z) return fail(MASE_ERR_ARG, "z is null");
  const Plan& p = c->plan;
  HIPTRY(hipMemcpyAsync((void*)c->d.z, z, sizeof(double) * (size_t)p.n_snap * p.n_meas,
                        hipMemcpyHostToDevice, c->stream));
  std::vector<double> wv(p.n_meas);
  for (int i = 0; i < p.n_meas; ++i) {
    wv[i] = w ? w[i] : 1.0 / (p.sigma[i] * p.sigma[i]);
    if (!(wv[i] >= 0.0) || !std::isfinite(wv[i])) return fail(MASE_ERR_ARG, "weights must be finite and >= 0");
  }
  HIPTRY(hipMemcpyAsync((void*)c->d.w, wv.data(), sizeof(double) * p.n_meas, hipMemcpyHostToDevice, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  c->have_z = true;
  return 0;
}

int mase_set_measurements_dev(mase_ctx* c, const double* z_dev, const double* w_dev) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!z_dev) return fail(MASE_ERR_ARG, "z_dev is null");
  const Plan& p = c->plan;
  HIPTRY(hipMemcpyAsync((void*)c->d.z, z_dev, sizeof(double) * (size_t)p.n_snap * p.n_meas,
                        hipMemcpyDeviceToDevice, c->stream));
  // NULL weights mean 1/sigma^2, as in mase_set_measurements
  HIPTRY(hipMemcpyAsync((void*)c->d.w, w_dev ? w_dev : c->w_default, sizeof(double) * p.n_meas,
                        hipMemcpyDeviceToDevice, c->stream));
  c->have_z = true;
  return 0;
}

int mase_set_state(mase_ctx* c, const double* vm, const double* va) {
  int rc = check_device(c);
  if (rc) return rc;
  if ((vm == nullptr) != (va == nullptr)) return fail(MASE_ERR_ARG, "give both vm and va or neither");
  const size_t n = (size_t)c->plan.n_snap * c->plan.n_bus;
  if (vm) {
    HIPTRY(hipMemcpyAsync(c->stage_vm, vm, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIPTRY(hipMemcpyAsync(c->stage_va, va, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIPTRY(launch_pack_state(c->d, c->stage_vm, c->stage_va, c->d.x, c->stream));
  } else {
    HIPTRY(launch_pack_state(c->d, nullptr, nullptr, c->d.x, c->stream));
  }
  HIPTRY(launch_reset_flags(c->d, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  for (int s = 0; s < c->plan.n_snap; ++s) c->h_active[s] = 1;
  return 0;
}

int mase_set_state_dev(mase_ctx* c, const double* vm_dev, const double* va_dev) {
  int rc = check_device(c);
  if (rc) return rc;
  if ((vm_dev == nullptr) != (va_dev == nullptr)) return fail(MASE_ERR_ARG, "give both vm and va or neither");
  HIPTRY(launch_pack_state(c->d, vm_dev, va_dev, c->d.x, c->stream));
  HIPTRY(launch_reset_flags(c->d, c->stream));
  for (int s = 0; s < c->plan.n_snap; ++s) c->h_active[s] = 1;
  return 0;
}

}  // extern "C"

namespace {

// One batched (or plain) iteration for every active snapshot, flags read
// back.  A snapshot that hits a non-positive pivot is frozen by k_update and
// reported through its status flags only, so callers can keep iterating the
// others.
int gn_iter_all(mase_ctx* c) {
  int rc = 0;
  const int S = c->plan.n_snap;
  int nactive_before = 0;
  for (int s = 0; s < S; ++s) nactive_before += c->h_active[s] != 0;
  if (c->opt.batched) {
    // event pairs recorded as graph nodes cannot be timed, so a profiled
    // iteration launches the same kernels directly on the stream
    if (c->opt.use_graph && !c->prof) {
      if (!c->gexec) {
        HIPTRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        rc = launch_batched_iteration(c, c->stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return fail(MASE_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        c->graph = g;
        HIPTRY(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
      }
      HIPTRY(hipGraphLaunch(c->gexec, c->stream));
    } else {
      if ((rc = launch_batched_iteration(c, c->stream))) return rc;
    }
    if ((rc = read_flags(c))) return rc;
    if ((rc = accumulate_profile(c, nactive_before))) return rc;
  } else {
    // plain schedule: snapshots one after another
    HIPTRY(hipMemcpyAsync(c->h_active, c->d.active, sizeof(int32_t) * S, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(hipStreamSynchronize(c->stream));
    std::vector<int32_t> act(c->h_active, c->h_active + S);
    for (int s = 0; s < S; ++s) {
      if (!act[s]) continue;
      if ((rc = launch_plain_iteration(c, s))) return rc;
    }
    if ((rc = read_flags(c))) return rc;
  }
  return 0;
}

}  // namespace

extern "C" {

int mase_gn_iter(mase_ctx* c, double* max_abs_dx) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!c->have_z) return fail(MASE_ERR_STATE, "no measurements set");
  if ((rc = gn_iter_all(c))) return rc;
  const int S = c->plan.n_snap;
  if (max_abs_dx) std::memcpy(max_abs_dx, c->h_maxdx, sizeof(double) * S);
  for (int s = 0; s < S; ++s)
    if (snapshot_bad(c, s))
      return fail(MASE_ERR_NOT_POSDEF, "non-positive pivot in snapshot " + std::to_string(s));
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner: candidate schedules timed on the context's own measurements.
// ---------------------------------------------------------------------------
namespace {

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Key of the tuning cache: the grid structure, partition, measurement set,
// batch size, boundary mode and the device.
std::string make_tune_key(const mase_ctx* c) {
  const Plan& p = c->plan;
  uint64_t h = 1469598103934665603ull;
  const int32_t dims[8] = {p.n_bus, p.n_branch, p.n_area, p.n_meas, p.n_snap, c->opt.gamma_mode,
                           c->opt.local_steps, c->area_lds ? 1 : 0};
  h = fnv1a(h, dims, sizeof(dims));
  h = fnv1a(h, p.br_from.data(), p.br_from.size() * sizeof(int32_t));
  h = fnv1a(h, p.br_to.data(), p.br_to.size() * sizeof(int32_t));
  h = fnv1a(h, p.bus_area.data(), p.bus_area.size() * sizeof(int32_t));
  h = fnv1a(h, p.meas_area.data(), p.meas_area.size() * sizeof(int32_t));
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) == hipSuccess) (void)hipGetDeviceProperties(&prop, dev);
  char buf[64];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  std::string arch(prop.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ' || ch == '\n') ch = '_';
  return std::string(buf) + "/" + (arch.empty() ? "unknown" : arch);
}

// One cache line per tuned configuration:
// "key npipe snode dense_mode dense_nb [elim_nt]" (elim_nt 0: per-class default).
bool read_tune_cache(const mase_ctx* c, int& npipe, int& snode, int& dmode, int& dnb, int& ent) {
  if (c->tune_path.empty()) return false;
  FILE* f = std::fopen(c->tune_path.c_str(), "r");
  if (!f) return false;
  char line[512], key[256];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    int a = 0, b = 0, m = 0, w = 0, e = 0;
    const int n = std::sscanf(line, "%255s %d %d %d %d %d", key, &a, &b, &m, &w, &e);
    if (n < 5) continue;
    if (n == 5) e = 0;
    if (c->tune_key == key && a >= 1 && (b == 0 || b == 1) && m >= DENSE_GLOBAL && m <= DENSE_WIDE && w >= 0 &&
        (e == 0 || e == 256 || e == 512 || e == 1024)) {
      npipe = a;
      snode = b;
      dmode = m;
      dnb = w;
      ent = e;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void write_tune_cache(const mase_ctx* c, int npipe, int snode, int dmode, int dnb, int ent) {
  if (c->tune_path.empty()) return;
  FILE* f = std::fopen(c->tune_path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d\n", c->tune_key.c_str(), npipe, snode, dmode, dnb, ent);
  std::fclose(f);
}

// Threads per workgroup of every LDS elimination class (0: each class's default).
void apply_elim_nt(mase_ctx* c, int nt) {
  c->elim_nt = nt;
  for (auto& cl : c->el_class)
    if (cl.nt) cl.nt = nt ? nt : cl.nt_default;
}

// Drops every captured graph (they bake in the schedule choices).
int reset_graphs(mase_ctx* c) {
  HIPTRY(hipStreamSynchronize(c->stream));
  if (c->pstream_area) HIPTRY(hipStreamSynchronize(c->pstream_area));
  for (auto st : c->pstream) HIPTRY(hipStreamSynchronize(st));
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  for (auto e : c->pgA) if (e) (void)hipGraphExecDestroy(e);
  for (auto e : c->pgB) if (e) (void)hipGraphExecDestroy(e);
  for (auto g : c->pgraphs) if (g) (void)hipGraphDestroy(g);
  for (auto e : c->pev_a) if (e) (void)hipEventDestroy(e);
  for (auto e : c->pev_b) if (e) (void)hipEventDestroy(e);
  for (auto st : c->pstream) if (st) (void)hipStreamDestroy(st);
  if (c->pstream_area) (void)hipStreamDestroy(c->pstream_area);
  c->pgA.clear();
  c->pgB.clear();
  c->pgraphs.clear();
  c->pev_a.clear();
  c->pev_b.clear();
  c->pstream.clear();
  c->pstream_area = nullptr;
  return 0;
}

// The batched iteration loop of mase_solve (pipelined when npipe > 1).
int solve_batched(mase_ctx* c, int max_iter) {
  const int S = c->plan.n_snap;
  int rc = read_flags(c);
  if (rc) return rc;
  if (c->opt.use_graph && !c->prof && c->npipe > 1) return pipelined_solve(c, max_iter);
  int nact = 0;
  for (int s = 0; s < S; ++s) nact += c->h_active[s] != 0;
  // a snapshot with a non-positive pivot is frozen by the update kernel;
  // the others keep iterating
  for (int it = 0; it < max_iter && nact > 0; ++it) {
    if ((rc = gn_iter_all(c))) return rc;
    nact = 0;
    for (int s = 0; s < S; ++s) nact += c->h_active[s] != 0;
  }
  return 0;
}

// Times two GN iterations of every candidate from the current state, keeps
// the fastest, restores the state.
int autotune(mase_ctx* c) {
  c->tuned = true;
  if (c->tune_key.empty()) c->tune_key = make_tune_key(c);
  // dense-block variants: the widest LDS panel that fits, a 32-column one,
  // and 16-column panels (each only where the create-time choice allows it)
  std::vector<std::pair<int, int>> dense_cands{{c->dense_mode, c->dense_nb}};
  if (c->dense_mode == DENSE_WIDE) {
    if (c->dense_nb > 32) dense_cands.push_back({DENSE_WIDE, 32});
    dense_cands.push_back({DENSE_PANEL16, 16});
  }
  int np = 0, sn = 0, dm = 0, dnb = 0, ent = 0;
  if (read_tune_cache(c, np, sn, dm, dnb, ent)) {
    int rc = reset_graphs(c);
    if (rc) return rc;
    c->npipe = std::max(1, std::min(np, c->plan.n_snap));
    c->gamma_snode = sn && c->snode_possible;
    apply_elim_nt(c, ent);
    for (const auto& dc : dense_cands)
      if (dc.first == dm && dc.second == dnb) {
        c->dense_mode = dm;
        c->dense_nb = dnb;
      }
    return 0;
  }
  const int S = c->plan.n_snap, K = c->plan.n_area;
  double2* sx = nullptr;
  int32_t* sflags = nullptr;
  double* smax = nullptr;
  const size_t nx = (size_t)S * c->plan.n_bus, nf = (size_t)S * (3 + K);
  int rc = dalloc(c, nx, &sx);
  if (!rc) rc = dalloc(c, nf, &sflags);
  if (!rc) rc = dalloc(c, (size_t)S, &smax);
  if (rc) return rc;
  auto save_restore = [&](bool save) -> int {
    const size_t bf = sizeof(int32_t) * S;
    double2* x = c->d.x;
    if (save) {
      HIPTRY(hipMemcpyAsync(sx, x, sizeof(double2) * nx, hipMemcpyDeviceToDevice, c->stream));
      HIPTRY(hipMemcpyAsync(sflags, c->d.active, bf, hipMemcpyDeviceToDevice, c->stream));
      HIPTRY(hipMemcpyAsync(sflags + S, c->d.iters, bf, hipMemcpyDeviceToDevice, c->stream));
      HIPTRY(hipMemcpyAsync(sflags + 2 * S, c->d.status, bf * (K + 1), hipMemcpyDeviceToDevice, c->stream));
      HIPTRY(hipMemcpyAsync(smax, c->d.maxdx, sizeof(double) * S, hipMemcpyDeviceToDevice, c->stream));
    } else {
      HIPTRY(hipMemcpyAsync(x, sx, sizeof(double2) * nx, hipMemcpyDeviceToDevice, c->stream));
      HIPTRY(hipMemcpyAsync(c->d.active, sflags, bf, hipMemcpyDeviceToDevice, c->stream));
      HIPTRY(hipMemcpyAsync(c->d.iters, sflags + S, bf, hipMemcpyDeviceToDevice, c->stream));
      HIPTRY(hipMemcpyAsync(c->d.status, sflags + 2 * S, bf * (K + 1), hipMemcpyDeviceToDevice, c->stream));
      HIPTRY(hipMemcpyAsync(c->d.maxdx, smax, sizeof(double) * S, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPTRY(hipStreamSynchronize(c->stream));
    return 0;
  };
  if ((rc = save_restore(true))) return rc;
  const bool snode0 = c->gamma_snode;
  double best = 1e300;
  int best_np = c->npipe, best_sn = snode0 ? 1 : 0;
  std::pair<int, int> best_dense{c->dense_mode, c->dense_nb};
  int best_ent = c->elim_nt;
  // a snapshot with a non-positive pivot only freezes itself, so a failure
  // here is a runtime error; the state and the schedule are restored on
  // every exit
  auto trials = [&]() -> int {
    for (int snc = 1; snc >= 0; --snc) {
      if (snc == 1 && !c->snode_possible) continue;
      for (int npc : {1, 2, 4, 8}) {
        if (npc > S) continue;
        for (const auto& dc : dense_cands) {
          int e = reset_graphs(c);
          if (e) return e;
          c->npipe = npc;
          c->gamma_snode = snc == 1;
          c->dense_mode = dc.first;
          c->dense_nb = dc.second;
          double t = 0.0;
          for (int rep = 0; rep < 2; ++rep) {  // the first run captures the graphs
            if ((e = save_restore(false))) return e;
            const auto t0 = std::chrono::steady_clock::now();
            if ((e = solve_batched(c, 2))) return e;
            HIPTRY(hipStreamSynchronize(c->stream));
            t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
          }
          if (t < best) {
            best = t;
            best_np = npc;
            best_sn = snc;
            best_dense = dc;
          }
        }
      }
    }
    // then the LDS elimination's workgroup size under the best schedule
    if (c->area_lds) {
      for (int ntc : {256, 512, 1024}) {
        int e = reset_graphs(c);
        if (e) return e;
        c->npipe = best_np;
        c->gamma_snode = best_sn == 1;
        c->dense_mode = best_dense.first;
        c->dense_nb = best_dense.second;
        apply_elim_nt(c, ntc);
        double t = 0.0;
        for (int rep = 0; rep < 2; ++rep) {
          if ((e = save_restore(false))) return e;
          const auto t0 = std::chrono::steady_clock::now();
          if ((e = solve_batched(c, 2))) return e;
          HIPTRY(hipStreamSynchronize(c->stream));
          t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (t < best) {
          best = t;
          best_ent = ntc;
        }
      }
    }
    return 0;
  };
  const int rc_trials = trials();
  const std::string err_trials = rc_trials ? g_err : std::string();
  rc = reset_graphs(c);
  c->npipe = best_np;
  c->gamma_snode = best_sn == 1;
  c->dense_mode = best_dense.first;
  c->dense_nb = best_dense.second;
  apply_elim_nt(c, best_ent);
  if (!rc) rc = save_restore(false);
  if (rc_trials) return fail(rc_trials, err_trials);
  if (rc) return rc;
  write_tune_cache(c, best_np, best_sn, best_dense.first, best_dense.second, best_ent);
  return 0;
}

}  // namespace

extern "C" {

int mase_solve(mase_ctx* c, double tol, int32_t max_iter, int32_t* iters, int32_t* converged) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!(tol > 0.0) || max_iter < 1) return fail(MASE_ERR_ARG, "need tol > 0 and max_iter >= 1");
  if (!c->have_z) return fail(MASE_ERR_STATE, "no measurements set");
  const int S = c->plan.n_snap;
  c->h_tol[0] = tol;
  HIPTRY(hipMemcpyAsync(c->dtol, c->h_tol, sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (c->opt.batched) {
    if (c->opt.autotune && !c->tuned && c->opt.use_graph && !c->prof)
      if ((rc = autotune(c))) return rc;
    if ((rc = solve_batched(c, max_iter))) return rc;
  } else {
    // plain schedule: one snapshot at a time, to convergence
    HIPTRY(hipMemcpyAsync(c->h_active, c->d.active, sizeof(int32_t) * S, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(hipStreamSynchronize(c->stream));
    std::vector<int32_t> act(c->h_active, c->h_active + S);
    for (int s = 0; s < S; ++s) {
      if (!act[s]) continue;
      for (int it = 0; it < max_iter; ++it) {
        if ((rc = launch_plain_iteration(c, s))) return rc;
        HIPTRY(hipMemcpyAsync(c->h_active + s, c->d.active + s, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HIPTRY(hipStreamSynchronize(c->stream));
        if (!c->h_active[s]) break;
      }
    }
    if ((rc = read_flags(c))) return rc;
  }
  HIPTRY(hipMemcpyAsync(c->h_iters, c->d.iters, sizeof(int32_t) * S, hipMemcpyDeviceToHost, c->stream));
  if ((rc = read_flags(c))) return rc;
  bool all = true, bad = false;
  for (int s = 0; s < S; ++s) {
    const bool b = snapshot_bad(c, s);
    const bool conv = !c->h_active[s] && !b;
    bad |= b;
    all &= conv;
    if (iters) iters[s] = c->h_iters[s];
    if (converged) converged[s] = conv ? 1 : 0;
  }
  if (bad) return fail(MASE_ERR_NOT_POSDEF, "a snapshot hit a non-positive pivot");
  return all ? MASE_OK : MASE_NOT_CONVERGED;
}

}  // extern "C"

namespace {

// Host-buffer ends of a stream solve: snapshots are uploaded chunk by chunk
// on a copy stream ahead of the stream position, and downloaded chunk by
// chunk once every snapshot of the chunk has left its slot.
struct StreamHost {
  const double* z_host = nullptr;   // [n_total][n_meas]
  const double* vm0_host = nullptr; // [n_total][n_bus] or null (flat start)
  const double* va0_host = nullptr;
  double* vm_host = nullptr;        // [n_total][n_bus]
  double* va_host = nullptr;
  double* z_dev = nullptr;          // device copies (workspace)
  double* vm0_dev = nullptr;
  double* va0_dev = nullptr;
  double* vm_dev = nullptr;
  double* va_dev = nullptr;
  hipStream_t cs = nullptr;         // copy stream (default priority)
  std::vector<hipEvent_t> up_ev;    // per uploaded chunk
  int64_t chunk = 64;
  int64_t up_to = 0;                // snapshots whose upload is enqueued
  int64_t down_to = 0;              // snapshots whose download is enqueued
  int64_t n_total = 0;
  int n_meas = 0, n_bus = 0;

  ~StreamHost() {
    for (auto e : up_ev) if (e) (void)hipEventDestroy(e);
    if (cs) (void)hipStreamDestroy(cs);
  }
  // enqueue uploads of every chunk that starts below `need` (and a little
  // ahead), then make `st` wait for the chunk that holds position need - 1
  int ensure(int64_t need, hipStream_t st) {
    need = std::min(need, n_total);
    const int64_t ahead = std::min(n_total, need + 2 * chunk);
    while (up_to < ahead) {
      const int64_t n = std::min(chunk, n_total - up_to);
      HIPTRY(hipMemcpyAsync(z_dev + up_to * n_meas, z_host + up_to * n_meas, sizeof(double) * n * n_meas,
                            hipMemcpyHostToDevice, cs));
      if (vm0_host) {
        HIPTRY(hipMemcpyAsync(vm0_dev + up_to * n_bus, vm0_host + up_to * n_bus, sizeof(double) * n * n_bus,
                              hipMemcpyHostToDevice, cs));
        HIPTRY(hipMemcpyAsync(va0_dev + up_to * n_bus, va0_host + up_to * n_bus, sizeof(double) * n * n_bus,
                              hipMemcpyHostToDevice, cs));
      }
      hipEvent_t e = nullptr;
      HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      up_ev.push_back(e);
      HIPTRY(hipEventRecord(e, cs));
      up_to += n;
    }
    if (need > 0) HIPTRY(hipStreamWaitEvent(st, up_ev[(size_t)((need - 1) / chunk)], 0));
    return 0;
  }
  // enqueue downloads of the chunks below `done` (whole chunks only unless
  // done == n_total), after the work recorded in `ev`
  int drain(int64_t done, hipEvent_t ev) {
    int64_t upto = done >= n_total ? n_total : done / chunk * chunk;
    if (upto <= down_to) return 0;
    HIPTRY(hipStreamWaitEvent(cs, ev, 0));
    const int64_t n = upto - down_to;
    HIPTRY(hipMemcpyAsync(vm_host + down_to * n_bus, vm_dev + down_to * n_bus, sizeof(double) * n * n_bus,
                          hipMemcpyDeviceToHost, cs));
    HIPTRY(hipMemcpyAsync(va_host + down_to * n_bus, va_dev + down_to * n_bus, sizeof(double) * n * n_bus,
                          hipMemcpyDeviceToHost, cs));
    down_to = upto;
    return 0;
  }
};

// Continuous batching core (mase_solve_stream and its host-buffer variant).
// The stream's device bookkeeping, grown on demand: slot tables (3 n_snap +
// 2 ints) and per-snapshot results (2 n_total ints).
int stream_buffers(mase_ctx* c, int64_t n_total, int32_t** tables, int32_t** results) {
  const int S = c->plan.n_snap;
  int rc = 0;
  if (!c->st_slots && (rc = dalloc(c, (size_t)3 * S + 2, &c->st_slots))) return rc;
  if (c->st_out_cap < n_total) {
    if (c->st_out) HIPTRY(hipFree(c->st_out));
    c->st_out = nullptr;
    c->st_out_cap = 0;
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(int32_t) * 2 * (size_t)n_total) != hipSuccess)
      return fail(MASE_ERR_OOM, "hipMalloc failed for the stream results");
    c->st_out = static_cast<int32_t*>(p);
    c->st_out_cap = n_total;
  }
  *tables = c->st_slots;
  *results = c->st_out;
  return 0;
}

// Continuous batching core.  tables [3 n_snap + 2] and results [2 n_total]
// are device ints the call owns for its duration.  no_alloc: allocate
// nothing (no graph instantiation, no autotuning, no host buffers): a graph
// already instantiated is replayed, else the kernels are launched directly.
int stream_solve(mase_ctx* c, const double* z_dev, const double* vm0_dev, const double* va0_dev, int64_t n_total,
                 double tol, int32_t max_iter, double* vm_dev, double* va_dev, int32_t* iters,
                 int32_t* converged, StreamHost* io, int32_t* tables, int32_t* results, bool no_alloc = false) {
  const int S = c->plan.n_snap;
  int rc = 0;
  int32_t* slot_id = tables;
  int32_t* retire = slot_id + S;
  int32_t* refill = retire + S;
  int32_t* next = refill + S;  // [0] stream position, [1] lowest position still in a slot
  int32_t* out_iters = results;
  int32_t* out_flag = results + n_total;
  const int32_t nt = (int32_t)n_total;
  c->h_tol[0] = tol;
  HIPTRY(hipMemcpyAsync(c->dtol, c->h_tol, sizeof(double), hipMemcpyHostToDevice, c->stream));
  // every slot idle, then the first refill loads the first n_snap snapshots
  HIPTRY(launch_stream_init(slot_id, next, S, c->stream));
  // weights: those of the last mase_set_measurements call, else 1/sigma^2
  if (!c->have_z)
    HIPTRY(hipMemcpyAsync((void*)c->d.w, c->w_default, sizeof(double) * c->plan.n_meas, hipMemcpyDeviceToDevice,
                          c->stream));
  // the first refill hands out positions [0, S), the first pass up to 2 S
  if (io && (rc = io->ensure(2 * (int64_t)S, c->stream))) return rc;
  HIPTRY(launch_stream_refill(c->d, slot_id, next, retire, refill, out_iters, out_flag, nt, max_iter, nullptr,
                              nullptr, c->stream));
  HIPTRY(launch_stream_copy(c->d, retire, refill, z_dev, vm0_dev, va0_dev, vm_dev, va_dev, c->stream));
  if ((rc = read_flags(c))) return rc;
  c->have_z = true;
  if (c->opt.autotune && !c->tuned && c->opt.use_graph && !c->prof && !no_alloc)
    if ((rc = autotune(c)) || (rc = read_flags(c))) return rc;
  // graph replay, or direct launches (profiling; or nothing may be allocated
  // and no graph exists yet)
  const bool use_graph = c->opt.use_graph && !c->prof && (!no_alloc || c->gexec);
  // while snapshots wait, every pass advances all S slots by one of at most
  // n_total * max_iter snapshot-iterations; after the last one has entered,
  // at most max_iter passes remain
  const int64_t limit = (n_total * max_iter + S - 1) / S + max_iter + 1;
  int32_t* hpos = c->h_st_pos;  // [2][2] pinned: next[0..1] of alternate passes
  // host_active / host_pos: where the refill kernel leaves the pass's active
  // flags and stream positions for the host (pinned buffers), or null
  auto launch_pass = [&](int32_t* host_active, int32_t* host_pos) -> int {
    if (use_graph) {
      if (!c->gexec) {
        HIPTRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        int e0 = launch_batched_iteration(c, c->stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (e0) { if (g) (void)hipGraphDestroy(g); return e0; }
        if (e != hipSuccess) return fail(MASE_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        c->graph = g;
        HIPTRY(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
      }
      HIPTRY(hipGraphLaunch(c->gexec, c->stream));
    } else {
      int e0 = launch_batched_iteration(c, c->stream);
      if (e0) return e0;
    }
    HIPTRY(launch_stream_refill(c->d, slot_id, next, retire, refill, out_iters, out_flag, nt, max_iter,
                                host_active, host_pos, c->stream));
    HIPTRY(launch_stream_copy(c->d, retire, refill, z_dev, vm0_dev, va0_dev, vm_dev, va_dev, c->stream));
    return 0;
  };
  auto count_active = [&](const int32_t* a) {
    int n = 0;
    for (int s = 0; s < S; ++s) n += a[s] != 0;
    return n;
  };
  int64_t known_next = S;  // stream position after the last pass whose flags were read
  if (use_graph || no_alloc) {
    // one pass always queued ahead: pass j + 1 is enqueued before the host
    // waits for the active flags of pass j (two pinned flag buffers, two
    // events), so the device never idles on the host's turnaround. A pass
    // enqueued after the stream has drained finds every slot idle and
    // changes nothing.
    auto enqueue = [&](int64_t j) -> int {
      // passes j - 1 and j may hand out up to 2 S positions past the last known one
      if (io && (rc = io->ensure(known_next + 2 * (int64_t)S, c->stream))) return rc;
      // the refill kernel leaves the active flags and stream positions in
      // the pinned buffers of this pass's parity
      if ((rc = launch_pass(c->h_st_active_dev + (j & 1) * S, c->h_st_pos_dev + 2 * (j & 1)))) return rc;
      HIPTRY(hipEventRecord(c->st_ev[j & 1], c->stream));
      return 0;
    };
    if (count_active(c->h_active) > 0) {
      if ((rc = enqueue(0))) return rc;
      for (int64_t j = 0;; ++j) {
        if (j + 1 > limit) {
          (void)hipStreamSynchronize(c->stream);
          return fail(MASE_ERR_STATE, "stream solve did not drain");
        }
        if ((rc = enqueue(j + 1))) return rc;
        HIPTRY(hipEventSynchronize(c->st_ev[j & 1]));
        if (io) {
          known_next = hpos[2 * (j & 1)];
          if ((rc = io->drain(hpos[2 * (j & 1) + 1], c->st_ev[j & 1]))) return rc;
        }
        if (count_active(c->h_st_active + (j & 1) * S) == 0) break;
      }
    }
    if ((rc = read_flags(c))) return rc;
  } else {
    int64_t pass = 0;
    for (;;) {
      const int nact = count_active(c->h_active);
      if (nact == 0) break;
      if (++pass > limit) return fail(MASE_ERR_STATE, "stream solve did not drain");
      if (io && (rc = io->ensure(known_next + (int64_t)S, c->stream))) return rc;
      if ((rc = launch_pass(nullptr, nullptr))) return rc;
      if ((rc = read_flags(c))) return rc;
      if ((rc = accumulate_profile(c, nact))) return rc;
      if (io) {
        HIPTRY(hipMemcpy(hpos, next, sizeof(int32_t) * 2, hipMemcpyDeviceToHost));
        known_next = hpos[0];
        HIPTRY(hipEventRecord(c->st_ev[0], c->stream));
        if ((rc = io->drain(hpos[1], c->st_ev[0]))) return rc;
      }
    }
  }
  if (io) {
    HIPTRY(hipEventRecord(c->st_ev[0], c->stream));
    if ((rc = io->drain(n_total, c->st_ev[0]))) return rc;
  }
  // per-snapshot results straight into the caller's arrays (converged holds
  // the outcome codes until they are turned into flags below; without it the
  // codes pass through a fixed buffer on the stack)
  if (iters) HIPTRY(hipMemcpyAsync(iters, out_iters, sizeof(int32_t) * n_total, hipMemcpyDeviceToHost, c->stream));
  bool all = true, bad = false;
  constexpr int64_t CH = 1024;
  int32_t buf[CH];
  for (int64_t i0 = 0; i0 < n_total; i0 += converged ? n_total : CH) {
    const int64_t n = converged ? n_total : std::min(CH, n_total - i0);
    int32_t* flags = converged ? converged : buf;
    HIPTRY(hipMemcpyAsync(flags, out_flag + i0, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; ++i) {
      const int32_t f = flags[i];
      bad |= f == 2;
      all &= f == 1;
      flags[i] = f == 1 ? 1 : 0;
    }
  }
  if (io) HIPTRY(hipStreamSynchronize(io->cs));
  if (bad) return fail(MASE_ERR_NOT_POSDEF, "a snapshot of the stream hit a non-positive pivot");
  return all ? MASE_OK : MASE_NOT_CONVERGED;
}

int stream_args(const mase_ctx* c, int64_t n_total, double tol, int32_t max_iter, const void* vm0, const void* va0) {
  if (!c->opt.batched) return fail(MASE_ERR_ARG, "the stream solve needs the batched schedule");
  if (!(tol > 0.0) || max_iter < 1) return fail(MASE_ERR_ARG, "need tol > 0 and max_iter >= 1");
  if (n_total < 0 || n_total > (int64_t(1) << 30)) return fail(MASE_ERR_ARG, "n_total must be in [0, 2^30]");
  if ((vm0 == nullptr) != (va0 == nullptr)) return fail(MASE_ERR_ARG, "give both vm0 and va0 or neither");
  return 0;
}

}  // namespace

extern "C" {

int mase_solve_stream(mase_ctx* c, const double* z_dev, const double* vm0_dev, const double* va0_dev,
                      int64_t n_total, double tol, int32_t max_iter, double* vm_dev, double* va_dev,
                      int32_t* iters, int32_t* converged) {
  int rc = check_device(c);
  if (rc) return rc;
  if ((rc = stream_args(c, n_total, tol, max_iter, vm0_dev, va0_dev))) return rc;
  if (n_total == 0) return MASE_OK;
  if (!z_dev || !vm_dev || !va_dev) return fail(MASE_ERR_ARG, "null z or output");
  int32_t *tables = nullptr, *results = nullptr;
  if ((rc = stream_buffers(c, n_total, &tables, &results))) return rc;
  return stream_solve(c, z_dev, vm0_dev, va0_dev, n_total, tol, max_iter, vm_dev, va_dev, iters, converged,
                      nullptr, tables, results);
}

int mase_solve_stream_noalloc(mase_ctx* c, const double* z_dev, const double* vm0_dev, const double* va0_dev,
                              int64_t n_total, double tol, int32_t max_iter, double* vm_dev, double* va_dev,
                              int32_t* iters, int32_t* converged) {
  int rc = check_device(c);
  if (rc) return rc;
  if ((rc = stream_args(c, n_total, tol, max_iter, vm0_dev, va0_dev))) return rc;
  if (n_total == 0) return MASE_OK;
  if (!z_dev || !vm_dev || !va_dev) return fail(MASE_ERR_ARG, "null z or output");
  const int64_t table_ints = 3 * (int64_t)c->plan.n_snap + 2;
  if (table_ints + 2 * n_total > NOALLOC_SCRATCH_INTS)
    return fail(MASE_ERR_ARG, "n_total = " + std::to_string(n_total) + " exceeds the no-alloc stream's limit of " +
                                  std::to_string(mase_stream_noalloc_max(c)) + " snapshots for this context");
  if (!c->noalloc_scratch) return fail(MASE_ERR_STATE, "scratch address not resolved");
  // tables first (k_stream_init clears what must start at zero), then the
  // results, which every snapshot writes once when it leaves its slot
  int32_t* tables = c->noalloc_scratch;
  int32_t* results = tables + table_ints;
  return stream_solve(c, z_dev, vm0_dev, va0_dev, n_total, tol, max_iter, vm_dev, va_dev, iters, converged,
                      nullptr, tables, results, /*no_alloc=*/true);
}

int64_t mase_stream_noalloc_max(const mase_ctx* c) {
  if (!c) return -1;
  return std::max<int64_t>(0, (NOALLOC_SCRATCH_INTS - (3 * (int64_t)c->plan.n_snap + 2)) / 2);
}

int64_t mase_stream_host_work(const mase_ctx* c, int64_t n_total, int32_t with_start) {
  if (!c || n_total < 0) return -1;
  const int64_t per = (int64_t)c->plan.n_meas + 2 * (int64_t)c->plan.n_bus * (with_start ? 2 : 1);
  return per * n_total;
}

int mase_solve_stream_host(mase_ctx* c, const double* z_host, const double* vm0_host, const double* va0_host,
                           int64_t n_total, double tol, int32_t max_iter, double* vm_host, double* va_host,
                           int32_t* iters, int32_t* converged, double* work_dev, int64_t work_len) {
  int rc = check_device(c);
  if (rc) return rc;
  if ((rc = stream_args(c, n_total, tol, max_iter, vm0_host, va0_host))) return rc;
  if (n_total == 0) return MASE_OK;
  if (!z_host || !vm_host || !va_host || !work_dev) return fail(MASE_ERR_ARG, "null z, output or workspace");
  if (work_len < mase_stream_host_work(c, n_total, vm0_host ? 1 : 0))
    return fail(MASE_ERR_ARG, "workspace smaller than mase_stream_host_work()");
  StreamHost io;
  io.n_total = n_total;
  io.n_meas = c->plan.n_meas;
  io.n_bus = c->plan.n_bus;
  io.chunk = std::max<int64_t>(1, c->plan.n_snap);
  io.z_host = z_host;
  io.vm0_host = vm0_host;
  io.va0_host = va0_host;
  io.vm_host = vm_host;
  io.va_host = va_host;
  double* w = work_dev;
  io.z_dev = w;
  w += n_total * (int64_t)io.n_meas;
  io.vm_dev = w;
  w += n_total * (int64_t)io.n_bus;
  io.va_dev = w;
  w += n_total * (int64_t)io.n_bus;
  if (vm0_host) {
    io.vm0_dev = w;
    w += n_total * (int64_t)io.n_bus;
    io.va0_dev = w;
  }
  HIPTRY(hipStreamCreateWithFlags(&io.cs, hipStreamNonBlocking));
  // the copy stream starts after everything queued so far on the context's stream
  HIPTRY(hipEventRecord(c->ev_main, c->stream));
  HIPTRY(hipStreamWaitEvent(io.cs, c->ev_main, 0));
  int32_t *tables = nullptr, *results = nullptr;
  if ((rc = stream_buffers(c, n_total, &tables, &results))) return rc;
  rc = stream_solve(c, io.z_dev, io.vm0_dev, io.va0_dev, n_total, tol, max_iter, io.vm_dev, io.va_dev, iters,
                    converged, &io, tables, results);
  (void)hipStreamSynchronize(io.cs);
  return rc;
}

int mase_state(mase_ctx* c, double* vm, double* va) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!vm || !va) return fail(MASE_ERR_ARG, "null output");
  const size_t n = (size_t)c->plan.n_snap * c->plan.n_bus;
  HIPTRY(launch_unpack_state(c->d, c->stage_vm, c->stage_va, c->stream));
  HIPTRY(hipMemcpyAsync(vm, c->stage_vm, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIPTRY(hipMemcpyAsync(va, c->stage_va, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  return 0;
}

int mase_state_dev(mase_ctx* c, double* vm_dev, double* va_dev) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!vm_dev || !va_dev) return fail(MASE_ERR_ARG, "null output");
  HIPTRY(launch_unpack_state(c->d, vm_dev, va_dev, c->stream));
  return 0;
}

int mase_objective(mase_ctx* c, double* J) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!J) return fail(MASE_ERR_ARG, "null output");
  if (!c->have_z) return fail(MASE_ERR_STATE, "no measurements set");
  const int K = c->plan.n_area, S = c->plan.n_snap;
  HIPTRY(launch_assemble(c->d, 0, K, 0, S, MODE_OBJECTIVE, c->lds_asm, c->br_lds, c->stream));
  std::vector<double> jp((size_t)S * K);
  HIPTRY(hipMemcpyAsync(jp.data(), c->d.jpart, sizeof(double) * jp.size(), hipMemcpyDeviceToHost, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  for (int s = 0; s < S; ++s) {
    double t = 0.0;
    for (int k = 0; k < K; ++k) t += jp[(size_t)s * K + k];
    J[s] = t;
  }
  return 0;
}

int mase_eval_h_dev(mase_ctx* c, const double* vm_dev, const double* va_dev, double* h_dev) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!vm_dev || !va_dev || !h_dev) return fail(MASE_ERR_ARG, "null argument");
  Dev d = c->d;
  HIPTRY(launch_pack_state(d, vm_dev, va_dev, c->xscratch, c->stream));
  d.x = c->xscratch;
  d.hout = h_dev;
  HIPTRY(launch_assemble(d, 0, c->plan.n_area, 0, c->plan.n_snap, MODE_EVAL_H, c->lds_asm, c->br_lds, c->stream));
  return 0;
}

int mase_profile(mase_ctx* c, int32_t enable) {
  int rc = check_device(c);
  if (rc) return rc;
  for (int i = 0; i < 2 * MASE_N_STAGE; ++i)
    if (!c->pev[i]) HIPTRY(hipEventCreate(&c->pev[i]));
  for (int i = 0; i < MASE_N_STAGE; ++i) {
    c->pms[i] = 0.0;
    c->plaunch[i] = 0;
    c->punits[i] = 0;
  }
  HIPTRY(hipStreamSynchronize(c->stream));
  c->prof = enable != 0;
  return 0;
}

int mase_profile_read(mase_ctx* c, double* total_ms, int64_t* launches, int64_t* units) {
  int rc = check_device(c);
  if (rc) return rc;
  for (int i = 0; i < MASE_N_STAGE; ++i) {
    if (total_ms) total_ms[i] = c->pms[i];
    if (launches) launches[i] = c->plaunch[i];
    if (units) units[i] = c->punits[i];
  }
  return 0;
}

int mase_info(const mase_ctx* c, int32_t what, int64_t* value) {
  if (!c || !value) return fail(MASE_ERR_ARG, "null argument");
  const Plan& p = c->plan;
  int64_t v = 0;
  switch (what) {
    case MASE_INFO_N_GAMMA: v = p.n_gamma_vars(); break;
    case MASE_INFO_N_BOUNDARY_BUS: v = (int64_t)p.gamma_bus.size(); break;
    case MASE_INFO_GAMMA_TAIL: v = p.sys[p.n_area].nt; break;
    case MASE_INFO_NNZ_FACTOR: v = p.vstride; break;
    case MASE_INFO_MAX_LEVELS: v = p.max_levels(); break;
    case MASE_INFO_FLOPS_LOCAL: v = (int64_t)p.flops_local(); break;
    case MASE_INFO_FLOPS_GAMMA: v = (int64_t)p.flops_gamma(); break;
    case MASE_INFO_BYTES_ASSEMBLY: v = (int64_t)p.bytes_assembly(); break;
    case MASE_INFO_N_SNAP: v = p.n_snap; break;
    case MASE_INFO_N_AREA: v = p.n_area; break;
    case MASE_INFO_BYTES_CONDENSE: v = (int64_t)p.bytes_condense(c->area_lds); break;
    case MASE_INFO_FLOPS_DENSE: v = (int64_t)p.flops_dense(); break;
    case MASE_INFO_BYTES_BACKSOLVE: v = (int64_t)p.bytes_backsolve(); break;
    case MASE_INFO_FLOPS_GAMMA_SPARSE: v = (int64_t)p.sys[p.n_area].elim_flops(); break;
    case MASE_INFO_GAMMA_LEVELS: v = p.sys[p.n_area].nlev; break;
    case MASE_INFO_GAMMA_SUPERNODES: v = (int64_t)p.sys[p.n_area].sn.size(); break;
    case MASE_INFO_GAMMA_SUPERNODAL: v = c->gamma_snode ? 1 : 0; break;
    case MASE_INFO_PIPELINE_GROUPS: v = c->npipe; break;
    case MASE_INFO_GAMMA_SUBTREE_GROUPS: v = c->d.n_sn_grp; break;
    case MASE_INFO_GAMMA_DENSE_PANEL: v = c->dense_mode == DENSE_WIDE ? c->dense_nb
                                        : c->dense_mode == DENSE_PANEL16 ? 16 : 0; break;
    case MASE_INFO_ELIM_THREADS: v = c->elim_nt; break;
    case MASE_INFO_AREA_LDS: {
      int n = 0;
      if (c->area_lds)
        for (int k = 0; k < p.n_area; ++k) n += p.tpl[k].lds_split > 0;
      v = n;
      break;
    }
    default: return fail(MASE_ERR_ARG, "unknown info key");
  }
  *value = v;
  return 0;
}

int mase_export_map(const mase_ctx* c, int32_t kind, int32_t area, int32_t* buf, int64_t cap,
                    int64_t* len) {
  if (!c || !len) return fail(MASE_ERR_ARG, "null argument");
  const Plan& p = c->plan;
  std::vector<int32_t> v;
  const bool per_area = kind >= MASE_MAP_LOCAL_VARS;
  if (per_area && (area < 0 || area >= p.n_area)) return fail(MASE_ERR_ARG, "area out of range");
  switch (kind) {
    case MASE_MAP_BOUNDARY_FLAG: v.assign(p.is_bnd.begin(), p.is_bnd.end()); break;
    case MASE_MAP_MEAS_AREA: v = p.meas_area; break;
    case MASE_MAP_GAMMA_VARS: v = canon_gamma_vars(p); break;
    case MASE_MAP_LOCAL_VARS: v = canon_local_vars(p, area); break;
    case MASE_MAP_N_INTERNAL: v.assign(1, canon_n_internal(p, area)); break;
    case MASE_MAP_E: v = canon_E(p, area); break;
    default: return fail(MASE_ERR_ARG, "unknown map kind");
  }
  *len = (int64_t)v.size();
  if (!buf || cap < (int64_t)v.size()) return fail(MASE_ERR_ARG, "buffer too small");
  std::copy(v.begin(), v.end(), buf);
  return 0;
}

int mase_export_pattern(const mase_ctx* c, int32_t area, int32_t* rowptr, int32_t* colidx, int64_t cap,
                        int64_t* nnz) {
  if (!c || !nnz) return fail(MASE_ERR_ARG, "null argument");
  if (area < 0 || area >= c->plan.n_area) return fail(MASE_ERR_ARG, "area out of range");
  std::vector<int32_t> rp, ci;
  canon_pattern(c->plan, area, rp, ci);
  *nnz = (int64_t)ci.size();
  if (!rowptr || !colidx || cap < (int64_t)ci.size()) return fail(MASE_ERR_ARG, "buffer too small");
  std::copy(rp.begin(), rp.end(), rowptr);
  std::copy(ci.begin(), ci.end(), colidx);
  return 0;
}

int mase_stage_assemble(mase_ctx* c) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!c->have_z) return fail(MASE_ERR_STATE, "no measurements set");
  HIPTRY(launch_assemble(c->d, 0, c->plan.n_area, 0, c->plan.n_snap, MODE_ASSEMBLE, c->lds_asm, c->br_lds, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  return 0;
}

int mase_stage_condense(mase_ctx* c) {
  int rc = check_device(c);
  if (rc) return rc;
  HIPTRY(launch_area_eliminate(c, 0, c->plan.n_area, 0, c->plan.n_snap, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  return 0;
}

int mase_stage_gamma_assemble(mase_ctx* c) {
  int rc = check_device(c);
  if (rc) return rc;
  const SysMeta& g = gsys(c);
  if (g.nn > 0) HIPTRY(launch_gamma_gather(c->d, 0, c->plan.n_snap, c->nslot_g, g.nn, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream));
  return 0;
}

int mase_stage_gamma_solve(mase_ctx* c) {
  int rc = check_device(c);
  if (rc) return rc;
  const SysMeta& g = gsys(c);
  const int K = c->plan.n_area, S = c->plan.n_snap;
  if (g.nn > 0) {
    if (g.ne > 0) HIPTRY(launch_gamma_sparse(c, 0, S, c->stream));
    HIPTRY(launch_dense_chol(c->d, 0, S, g.ld, c->dense_mode, c->dense_nb, c->stream));
    if (g.ne > 0) HIPTRY(launch_gamma_back(c, 0, S, c->stream));
  }
  HIPTRY(hipStreamSynchronize(c->stream));
  return 0;
}

int mase_stage_update(mase_ctx* c, double* max_abs_dx) {
  int rc = check_device(c);
  if (rc) return rc;
  HIPTRY(launch_area_backsolve(c, 0, c->plan.n_area, 0, c->plan.n_snap, c->stream));
  HIPTRY(launch_update(c->d, 0, c->plan.n_snap, c->stream));
  if ((rc = read_flags(c))) return rc;
  if (max_abs_dx) std::memcpy(max_abs_dx, c->h_maxdx, sizeof(double) * c->plan.n_snap);
  for (int s = 0; s < c->plan.n_snap; ++s)
    if (snapshot_bad(c, s)) return fail(MASE_ERR_NOT_POSDEF, "non-positive pivot");
  return 0;
}

int mase_read_local_system(mase_ctx* c, int32_t snap, int32_t area, double* G, double* b) {
  int rc = check_device(c);
  if (rc) return rc;
  const Plan& p = c->plan;
  if (snap < 0 || snap >= p.n_snap || area < 0 || area >= p.n_area || !G || !b)
    return fail(MASE_ERR_ARG, "bad argument");
  const SysPlan& s = p.sys[area];
  std::vector<double> vals(s.nval), rhs(2 * (size_t)s.nn);
  HIPTRY(hipMemcpy(vals.data(), c->d.vals + (size_t)snap * p.vstride + p.val_off[area],
                   sizeof(double) * s.nval, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(rhs.data(), c->d.rhs + (size_t)snap * p.rstride + p.rhs_off[area],
                   sizeof(double) * rhs.size(), hipMemcpyDeviceToHost));
  if (c->area_lds && p.tpl[area].lds_split > 0) {
    // the assembly wrote the compact blocks below the LDS split (fill
    // positions there are zero) and the packed storage above it
    const AreaTemplates& t = p.tpl[area];
    std::vector<double> gc(4 * t.cimg.size() + 1);
    if (!t.cimg.empty())
      HIPTRY(hipMemcpy(gc.data(), c->d.vals + (size_t)snap * p.vstride + p.gc_off[area],
                       sizeof(double) * 4 * t.cimg.size(), hipMemcpyDeviceToHost));
    std::fill(vals.begin(), vals.begin() + t.lds_split, 0.0);
    for (size_t i = 0; i < t.cimg.size(); ++i)
      for (int e = 0; e < 4; ++e) vals[(size_t)t.cimg[i] + e] = gc[4 * i + e];
  }
  const std::vector<int32_t> ci = canon_index(p, area);
  int dim = 0;
  for (int32_t v : ci) dim += v >= 0;
  std::fill(G, G + (size_t)dim * dim, 0.0);
  unpack_blocks(p, area, vals, ci, dim, 0, [](int) { return true; }, G);
  for (int v = 0; v < 2 * s.nn; ++v)
    if (ci[v] >= 0) b[ci[v]] = rhs[v];
  return 0;
}

int mase_read_schur(mase_ctx* c, int32_t snap, int32_t area, double* S, double* bhat) {
  int rc = check_device(c);
  if (rc) return rc;
  const Plan& p = c->plan;
  if (snap < 0 || snap >= p.n_snap || area < 0 || area >= p.n_area || !S || !bhat)
    return fail(MASE_ERR_ARG, "bad argument");
  const SysPlan& s = p.sys[area];
  std::vector<double> vals(s.nval), rhs(2 * (size_t)s.nn);
  HIPTRY(hipMemcpy(vals.data(), c->d.vals + (size_t)snap * p.vstride + p.val_off[area],
                   sizeof(double) * s.nval, hipMemcpyDeviceToHost));
  HIPTRY(hipMemcpy(rhs.data(), c->d.rhs + (size_t)snap * p.rstride + p.rhs_off[area],
                   sizeof(double) * rhs.size(), hipMemcpyDeviceToHost));
  const std::vector<int32_t> ci = canon_index(p, area);
  const int off = canon_n_internal(p, area);
  int dim = 0;
  for (int v = 2 * s.ne; v < 2 * s.nn; ++v) dim += ci[v] >= 0;
  std::fill(S, S + (size_t)dim * dim, 0.0);
  const int ne = s.ne;
  unpack_blocks(p, area, vals, ci, dim, off, [ne](int i) { return i >= ne; }, S);
  for (int v = 2 * s.ne; v < 2 * s.nn; ++v)
    if (ci[v] >= 0) bhat[ci[v] - off] = rhs[v];
  return 0;
}

int mase_read_gamma_system(mase_ctx* c, int32_t snap, double* S, double* bhat) {
  int rc = check_device(c);
  if (rc) return rc;
  const Plan& p = c->plan;
  if (snap < 0 || snap >= p.n_snap || !S || !bhat) return fail(MASE_ERR_ARG, "bad argument");
  const int K = p.n_area;
  const SysPlan& s = p.sys[K];
  std::vector<double> vals(std::max(1, s.nval)), rhs(std::max<size_t>(1, 2 * (size_t)s.nn));
  if (s.nval) HIPTRY(hipMemcpy(vals.data(), c->d.vals + (size_t)snap * p.vstride + p.val_off[K],
                               sizeof(double) * s.nval, hipMemcpyDeviceToHost));
  if (s.nn) HIPTRY(hipMemcpy(rhs.data(), c->d.rhs + (size_t)snap * p.rstride + p.rhs_off[K],
                             sizeof(double) * 2 * s.nn, hipMemcpyDeviceToHost));
  const std::vector<int32_t> ci = canon_index(p, K);
  const int dim = p.n_gamma_vars();
  std::fill(S, S + (size_t)dim * dim, 0.0);
  unpack_blocks(p, K, vals, ci, dim, 0, [](int) { return true; }, S);
  for (int v = 0; v < 2 * s.nn; ++v)
    if (ci[v] >= 0) bhat[ci[v]] = rhs[v];
  return 0;
}

int mase_read_step(mase_ctx* c, int32_t snap, double* dx) {
  int rc = check_device(c);
  if (rc) return rc;
  const Plan& p = c->plan;
  if (snap < 0 || snap >= p.n_snap || !dx) return fail(MASE_ERR_ARG, "bad argument");
  std::vector<double> rhs(p.rstride);
  HIPTRY(hipMemcpy(rhs.data(), c->d.rhs + (size_t)snap * p.rstride, sizeof(double) * p.rstride,
                   hipMemcpyDeviceToHost));
  for (int b = 0; b < p.n_bus; ++b) {
    const int src = p.bus_dx_src[b];
    dx[2 * b] = (b == p.slack) ? 0.0 : rhs[src];
    dx[2 * b + 1] = rhs[src + 1];
  }
  return 0;
}

}  // extern "C"
