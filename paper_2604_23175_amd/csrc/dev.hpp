// Device-resident plan and per-iteration buffers shared by the kernels and
// the host API.  All arrays are flattened over systems (areas 0..K-1, the
// boundary system K); index fields inside records are already rebased to the
// flattened arrays.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mase {

// Per system (area or boundary system).
struct SysMeta {
  int32_t nn, ne, nt, ld;         // buses, eliminated, tail, tail leading dim
  int32_t tail_off, nval, pin_off, nlev;
  int32_t val_off, rhs_off;       // offsets inside one snapshot's value / rhs block
  int32_t cd_ptr, up_ptr, rb_ptr, bs_ptr;  // first entry of this system's level pointers
  int32_t gbus;                   // first entry of local->global bus map
  int32_t asm_pin;                // offset the assembly writes the pinned slack block to, or -1
};

// Per area templates (Section 4.1).
struct AreaMeta {
  int32_t nn, nbr, nrow, nslot;
  int32_t br, inc_ptr, row, slot;  // first entries in the flattened arrays
  int32_t rslot, tail_src, slack_local;
  int32_t stage_off;  // doubles: this area's region in a snapshot's assembly staging (global mode)
  // elimination in LDS: compact G at val_off + gc_rel (n_cslot blocks, their
  // packed offsets from cimg), packed storage [0, split) held in LDS
  int32_t gc_rel, n_cslot, cimg, split;
};

enum { MODE_ASSEMBLE = 0, MODE_OBJECTIVE = 1, MODE_EVAL_H = 2 };

struct Dev {
  // sizes
  int32_t n_bus, n_meas, n_area, n_snap, slack;
  int32_t bs_max_nn_area, bs_max_nn_gamma;  // largest local bus counts (back substitution LDS)
  int64_t vstride, rstride;
  // plan
  const SysMeta* sys;
  const AreaMeta* area;
  const int32_t* area_order;
  const int32_t* gbus;
  const int32_t *br_lf, *br_lt;
  const double *br_g, *br_bs, *br_hb;
  const int32_t *inc_ptr, *inc_end;
  const int32_t *row_type, *row_loc, *row_meas;
  const int4* rowrec;  // per area row: {type, loc, meas, 0}
  const int4* slot;
  const int4* scon;   // per G-slot contribution: {type, loc, meas, role_p | role_q << 16}
  const int4* rslot;  // per area rhs item: {cbeg, cend, local bus, 0}
  const int32_t* slot_rhs;  // per slot: rhs offset 2 v of a diagonal slot (v, v), else -1
  const int4* rcon;   // per rhs contribution: {type, loc, meas, role}
  const int32_t *cd_ptr, *up_ptr, *rb_ptr, *bs_ptr;
  const int32_t* bs_lg;  // parallel to bs_ptr: log2 of the lanes per column of each level
  const int4* cd_items;
  const int4* up_tgt;
  const int2* up_con;
  const int4* rb_tgt;
  const int2* rb_con;
  const int4* bs_items;
  const int2* bs_con;
  // the same update / rhs lists addressed by packed offsets (elimination in LDS)
  const int4* up_tgt_img;
  const int2* up_con_img;
  const int2* rb_con_img;
  const int32_t* cimg;   // per compact G block: its packed offset
  // supernodes of the boundary system (the plan's sn, sn2, sn_rows, sn_tgt)
  int32_t n_sn;
  const int4* sn;
  const int4* sn2;
  const int32_t* sn_rows;
  const int32_t* sn_tgt;
  // elimination subtree groups (one workgroup each) and tail rows of the panels
  int32_t n_sn_grp;
  const int32_t* sn_grp_ptr;
  const int32_t* sn_grp;
  const int4* sn3;
  int32_t n_tail_ent;
  const int4* tail_ent;
  const int32_t* tail_con;
  double* sn_tl;       // [n_snap][tl_stride]: every supernode's U_q and c_q
  int32_t tl_stride;
  const int4* g_slot;
  const int4* g_con;
  const int2* g_rslot;
  const int32_t* g_rcon;
  const int32_t* tail_src;
  const int32_t* bus_dx_src;
  // measurements
  const double* z;  // [n_snap][n_meas]
  const double* w;  // [n_meas]
  // state and work buffers
  double2* x;       // [n_snap][n_bus] (theta, |V|)
  double* vals;     // [n_snap][vstride]
  double* rhs;      // [n_snap][rstride]
  double* jpart;    // [n_snap][n_area]
  double* hout;     // [n_snap][n_meas] (MODE_EVAL_H)
  int32_t* active;  // [n_snap]
  int32_t* iters;   // [n_snap]
  int32_t* status;  // [n_snap][n_area + 1]: 1 = non-positive pivot
  double* maxdx;    // [n_snap]
  const double* tol;  // [1]
  // assembly staging in HBM for areas too large for LDS: per snapshot
  // asm_stride doubles, area k's states, cos/sin and injection data at
  // AreaMeta::stage_off (nullptr: staging in LDS)
  double* asm_stage;
  int64_t asm_stride;
  // 1: the assembly stages its rows' weights and measurements in LDS
  int32_t asm_wz;
};

}  // namespace mase
