// Host-side setup of the multi-area estimator: maps, orderings, symbolic
// factorisation, level schedules and contribution lists.  Everything here is
// integer work done once per topology (arXiv 2604.23175, Section 4.1: the
// sparsity structure is decoupled from the values and built once; Section
// 4.3: the factorisation pattern is built once, values are refreshed per
// iteration).  The result is a Plan that the device side copies to HBM.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace mase {

struct I2 { int32_t x, y; };
struct I4 { int32_t x, y, z, w; };

// Roles of a support entry of a measurement row (see AreaTemplates).
constexpr int ROLE_SELF = 0xFFFF;   // the row's own bus (injection bus, flow's measured end, |V| bus)
constexpr int ROLE_OTHER = 0xFFFE;  // the unmeasured end of a flow row's branch
constexpr int MAX_LOCAL_BRANCH = 0xFFF0;
// Flag in an update target's stride: the target has exactly one contribution.
constexpr int32_t UP_SINGLE = 1 << 30;
// LDS budget (doubles) for staging one schedule step of the elimination.
constexpr int LDS_STAGE_DOUBLES = 6144;
// Widest supernode (buses): its panel is at most 64 variables wide.
constexpr int SN_MAX_W = 32;
// Workgroup sizes the back substitution's lane groups are chosen for (areas,
// boundary system).
constexpr int BS_THREADS_AREA = 256;
constexpr int BS_THREADS_GAMMA = 1024;
// LDS of one workgroup on gfx950 (doubles): the budget for holding an area's
// whole packed storage (or all but its Schur block) during its elimination.
constexpr int AREA_LDS_DOUBLES = 160 * 1024 / 8;

// Panel geometry of a supernode of w buses with r row buses below: the LDS
// panel has sn_rows_padded() rows (the 2w own variables padded to a multiple
// of 16, then the 2r row variables padded likewise) and sn_cols_padded()
// columns, column-major with pitch rows + 1; after it the rhs, the Schur
// target table and the r row bus ids.
inline int sn_cols_padded(int w) { return (2 * w + 15) / 16 * 16; }
inline int sn_rows_padded(int w, int r) { return sn_cols_padded(w) + (2 * r + 15) / 16 * 16; }
inline int sn_lds_bytes_of(int w, int r) {
  const int M = sn_rows_padded(w, r);
  return 8 * ((M + 1) * sn_cols_padded(w) + M) + 4 * (r * (r + 1) / 2) + 4 * r;
}

// One symmetric positive definite system over "buses" (2x2 blocks: theta, |V|)
// eliminated by the level-scheduled sparse engine.  Local buses [0, ne) are
// eliminated in order; [ne, nn) form the dense trailing ("tail") block.
//
// Packed value storage (doubles), per snapshot:
//   for each eliminated bus j: diagonal block (4 doubles, column-major 2x2)
//   followed by one 2x2 block per row bus i in strct[j] (column-major);
//   then the tail: a dense column-major matrix with leading dimension ld
//   (ld = 2*nt rounded up to 16), of which the lower triangle is used, or
//   with packed_tail its lower triangle of 2x2 blocks, each contiguous.
// Right-hand side storage: 2 doubles per local bus.
struct SysPlan {
  int nn = 0, ne = 0, nt = 0;
  std::vector<int> gbus;                 // local bus -> global bus
  std::vector<std::vector<int>> strct;   // eliminated bus j -> sorted local rows i > j
  std::vector<int32_t> col_off;          // eliminated bus j -> offset of its diagonal block
  int32_t tail_off = 0;
  int32_t ld = 0;                        // tail leading dimension (multiple of 16)
  // Packed tail (the areas' Schur blocks): the lower triangle of 2x2 blocks,
  // each block contiguous (column-major 2x2), block columns one after another;
  // else (the boundary system) the dense column-major ld x ld layout above.
  bool packed_tail = false;
  int32_t nval = 0;                      // doubles of packed storage
  int32_t pin_off = -1;                  // entry forced to 1 (slack theta pivot), or -1
  std::vector<int> level;                // eliminated bus -> level (leaves 0)
  int nlev = 0;

  // Level schedule (all offsets relative to this system's value / rhs base).
  // The blocks L_ij a level computes and its y_j are also staged in LDS; the
  // update lists address them by LDS double offsets ("slots").
  std::vector<int32_t> cd_ptr;  // [nlev+1] -> cd_items
  std::vector<I4> cd_items;     // {diag_off, blk_off (-1: the diagonal item), rhs_j, LDS slot}
  std::vector<int32_t> up_ptr;  // [nlev+1] -> up_tgt
  std::vector<I4> up_tgt;       // {tgt_off, tgt_stride [| UP_SINGLE], cbeg, cend} or, with
                                // UP_SINGLE, {tgt_off, stride, slot L_ij, slot L_pj}
  std::vector<I2> up_con;       // {slot L_ij, slot L_pj}: target -= L_ij * L_pj^T
  std::vector<int32_t> rb_ptr;  // [nlev+1] -> rb_tgt
  std::vector<I4> rb_tgt;       // {rhs_i, cbeg, cend, 0}
  std::vector<I2> rb_con;       // {slot L_ij, slot y_j}: y_i -= L_ij * y_j
  int32_t lds_doubles = 0;      // LDS staging needed by the largest level
  // Supernodes of the eliminated buses (built for the boundary system): runs
  // of consecutive buses j, j+1, ... in which each bus is the elimination-tree
  // parent of the previous one and the structures nest, strct[j] = {j+1} U
  // strct[j+1], at most SN_MAX_W buses wide.  Such a run is one dense panel:
  // its columns are contiguous in the packed storage, and its rows below the
  // diagonal block are the same bus list R for every column.
  std::vector<I4> sn;             // {first bus c0, width w, |R| = r, base of R in sn_rows}
  std::vector<I4> sn2;            // {offset of column c0's diagonal block, doubles of the
                                  // panel's columns (contiguous), base in sn_tgt,
                                  // number of R buses in the tail}
  std::vector<int32_t> sn_tbase;  // [nsn+1] -> sn_tgt
  std::vector<int32_t> sn_rows;   // R of each supernode, ascending local bus ids
  std::vector<int32_t> sn_tgt;    // per supernode, for a >= c in R: offset of block (R[a], R[c])
                                  // at a(a+1)/2 + c (in the dense tail when >= tail_off)
  int32_t sn_lds_bytes = 0;       // LDS of the largest panel (values, rhs, target offsets)
  // Elimination subtrees: a supernode's parent is the supernode holding R[0];
  // one whose R is empty or starts in the tail is a root.  Subtrees of
  // different roots share no factor entries outside the tail block and the
  // tail rhs, so they are eliminated in parallel (one workgroup per group of
  // roots) and their updates of the tail are applied afterwards, per target
  // in supernode order.
  std::vector<int32_t> sn_root;   // supernode -> root of its subtree
  std::vector<double> sn_cost;    // estimated elimination time of the supernode (arbitrary unit)
  std::vector<int32_t> sn_grp_ptr;  // [ngrp+1] -> sn_grp
  std::vector<int32_t> sn_grp;      // supernodes of each group, ascending
  // The tail updates of each supernode, U_q = L_T L_T^T over its tail rows T
  // (2 ntail of them, column-major 2 ntail x 2 ntail) and c_q = -L_T y_q, go to
  // a per-snapshot buffer; each tail entry then gathers its contributions in
  // supernode order.
  std::vector<I4> sn3;            // {offset of U_q, offset of c_q, 0, 0} in that buffer
  std::vector<I4> tail_ent;       // {target, 0 matrix (col * ld + row) / 1 rhs (variable), cbeg, cend}
  std::vector<int32_t> tail_con;  // buffer offsets, per target in supernode order
  int32_t tl_doubles = 0;         // doubles of the compact buffer per snapshot
  // The same update and rhs lists for a system held whole in LDS: factor
  // blocks are addressed by their packed-storage offsets instead of staging
  // slots (a single-contribution target carries the two offsets inline), and
  // y_j by its rhs offset 2 j.
  std::vector<I4> up_tgt_img;   // parallel to up_tgt
  std::vector<I2> up_con_img;   // {off L_ij, off L_pj}
  std::vector<I2> rb_con_img;   // {off L_ij, rhs offset of y_j}
  std::vector<int32_t> bs_ptr;  // [nlev+1] -> bs_items (same levels, run top-down)
  std::vector<I4> bs_items;     // {diag_off, rhs_j, cbeg, cend}
  std::vector<I2> bs_con;       // {off L_ij, rhs_i}: t -= L_ij^T * x_i
  // [nlev+1] (last entry unused): log2 of the lanes that share one column of
  // a level in the back substitution (1..64 lanes; the sum over the column's
  // rows is split over them), chosen per level for the fewest rounds of
  // dependent loads: many short columns near the leaves, few long ones near
  // the root
  std::vector<int32_t> bs_lg;

  void build_supernodes();               // fills sn*, after the schedule
  void group_supernodes(int max_groups); // sn_grp*: roots packed into at most max_groups groups
  int32_t blk_off(int i, int j) const;   // block (i, j), i >= j
  int32_t blk_stride(int i, int j) const;
  double elim_flops() const;             // flops of eliminating [0, ne) with rhs
};

// Measurement templates of one area (Section 4.1): structure-of-arrays rows
// and the static index maps that let the assembly kernel evaluate residuals
// and partials and sum their contributions into the packed G^k and b^k.
struct AreaTemplates {
  // local branches (at least one end in the area)
  std::vector<int32_t> br_lf, br_lt;       // local bus of the from / to end
  std::vector<double> br_g, br_bs, br_hb;  // series conductance, susceptance, half charging
  std::vector<int32_t> br_gid;             // global branch id
  // per local bus: incident local branch ends (own buses only), encoded
  // (branch << 1) | side, side 0 = the bus is the from end
  std::vector<int32_t> inc_ptr, inc_end;
  // rows owned by the area
  std::vector<int32_t> row_type, row_loc, row_meas;  // loc: local bus or local branch
  // G slots in packed order: {offset, stride, cbeg, cend} (stride < 0 marks a
  // diagonal block, kept exactly symmetric) and contributions
  // {row, role_p | role_q << 16}: slot += w * h_p h_q^T
  std::vector<I4> slot;
  std::vector<I2> scon;
  // rhs per local bus: {cbeg, cend} and contributions {row, role}
  std::vector<I2> rslot;
  std::vector<I2> rcon;
  int64_t n_contrib() const { return (int64_t)scon.size() + (int64_t)rcon.size(); }
  // Output of the assembly for the elimination that holds the area in LDS:
  // the slots with at least one contribution below lds_split go to a compact
  // array (4 doubles each, in this order; cslot offsets count from its start,
  // cimg gives each one's offset in the packed storage); fill positions there
  // are zeroed in LDS instead of being written.  Slots at or above lds_split
  // (the Schur block, when the area does not fit whole) keep their
  // packed-storage offsets in tslot and are all written, fill included.
  std::vector<I4> cslot, tslot;
  std::vector<int32_t> cimg;
  int32_t lds_split = 0;   // doubles of the packed storage held in LDS (0: does not fit;
                           // the area then runs the level engine over HBM)
};

struct Input {
  int32_t n_bus, n_branch;
  const int32_t *br_from, *br_to;
  const double *br_r, *br_x, *br_b;
  int32_t slack, n_area;
  const int32_t* bus_area;
  int32_t n_meas;
  const int32_t *meas_type, *meas_at;
  const double* meas_sigma;
  int32_t n_snap;
  int32_t gamma_mode;
};

struct Plan {
  int n_bus = 0, n_branch = 0, n_area = 0, n_meas = 0, slack = 0, n_snap = 0;
  std::vector<int32_t> br_from, br_to;
  std::vector<double> sigma;
  std::vector<int32_t> bus_area;
  std::vector<char> is_bnd;
  std::vector<int32_t> meas_area;
  std::vector<int32_t> gamma_bus;         // boundary buses, ascending id (canonical Gamma)
  std::vector<int32_t> gamma_canon_pos;   // bus -> position in gamma_bus or -1

  // systems 0..n_area-1 are the areas, system n_area is the boundary system
  std::vector<SysPlan> sys;
  std::vector<AreaTemplates> tpl;
  std::vector<std::vector<int32_t>> local_of_bus;  // per area: bus -> local index or -1

  // per-snapshot layout (doubles)
  std::vector<int32_t> val_off, rhs_off;  // per system
  std::vector<int32_t> gc_off;            // per area: the compact G array (after all systems)
  int64_t vstride = 0, rstride = 0;
  bool lds_areas = false;                 // some area fits the LDS budget (its elimination in LDS)

  // boundary assembly (Eq. 11): Gamma slots {offset, stride, cbeg, cend},
  // contributions {src_off, src_ld, transpose, 0} (offsets relative to the
  // snapshot's value base); rhs per Gamma local bus {cbeg, cend} with
  // contributions = source rhs offsets
  std::vector<I4> g_slot, g_con;
  std::vector<I2> g_rslot;
  std::vector<int32_t> g_rcon;
  // per area tail bus: rhs offset of the same bus in the boundary system
  std::vector<int32_t> tail_src;      // flattened, per area at tail_src_ptr[k]
  std::vector<int32_t> tail_src_ptr;  // [n_area+1]
  // per bus: rhs offset (relative to snapshot rhs base) holding its dx
  std::vector<int32_t> bus_dx_src;
  // area order for launches: longest elimination first, balanced over the
  // 8 chiplets when the area count is a multiple of 8
  std::vector<int32_t> area_order;

  int max_levels() const;
  double flops_local() const;
  double flops_gamma() const;
  double bytes_assembly() const;  // algorithmic HBM bytes per snapshot (nonzero G blocks only)
  // read G once, write L once (areas), rhs; lds: areas that fit are eliminated in LDS
  double bytes_condense(bool lds) const;
  double bytes_backsolve() const; // areas: read L once, rhs read / write
  double flops_dense() const;     // dense boundary block of n = 2 nt variables: n^3/3 + 2 n^2
  int n_gamma_vars() const;
};

// Builds the plan; returns "" on success or an error message (bad input).
std::string build_plan(const Input& in, Plan& plan);

// Canonical exports (see mase.h).
std::vector<int32_t> canon_local_vars(const Plan& p, int area);
int canon_n_internal(const Plan& p, int area);
std::vector<int32_t> canon_gamma_vars(const Plan& p);
std::vector<int32_t> canon_E(const Plan& p, int area);
void canon_pattern(const Plan& p, int area, std::vector<int32_t>& rowptr,
                   std::vector<int32_t>& colidx);

}  // namespace mase
