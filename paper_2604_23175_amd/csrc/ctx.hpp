// Context of the C ABI (mase_ctx), shared by api.hip and mlp.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dev.hpp"
#include "mase.h"
#include "plan.hpp"

struct mase_ctx {
  mase::Plan plan;
  mase_options opt{};
  bool host_only = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<hipStream_t> astreams;
  std::vector<hipEvent_t> aevents;
  hipEvent_t ev_main = nullptr;
  mase::Dev d{};
  std::vector<void*> dallocs;
  double2* xscratch = nullptr;
  double* stage_vm = nullptr;
  double* stage_va = nullptr;
  double* dtol = nullptr;
  double* w_default = nullptr;  // 1/sigma^2 per measurement (device)
  size_t lds_asm = 0;
  bool br_lds = false;
  size_t lds_el_area = 0, lds_el_gamma = 0;  // elimination staging LDS bytes
  // the areas' elimination held in LDS: launch classes over runs of
  // area_order positions with the same workgroups per CU (LDS bytes of the
  // largest area in the run, threads per workgroup, Schur block in HBM)
  bool area_lds = false;
  struct ElClass { int a0, na; size_t lds; int nt; bool tail_hbm; int nt_default; };
  std::vector<ElClass> el_class;
  int elim_nt = 0;  // threads per LDS elimination workgroup for every class (0: class defaults)
  int dense_mode = 0;                         // DENSE_GLOBAL / DENSE_PANEL16 / DENSE_WIDE
  int dense_nb = 16;                          // panel width of DENSE_WIDE
  bool gamma_snode = false;                   // supernodal boundary elimination
  size_t lds_sn = 0;                          // its LDS bytes
  int nslot_g = 0;
  bool have_z = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // pipelined solve: snapshot groups [pg_s0[g], pg_s0[g+1]) iterate on their
  // own streams; area stages of all groups share pstream_area
  int npipe = 1;
  std::vector<int> pg_s0;
  hipStream_t pstream_area = nullptr;
  std::vector<hipStream_t> pstream;
  std::vector<hipEvent_t> pev_a, pev_b;
  std::vector<hipGraph_t> pgraphs;
  std::vector<hipGraphExec_t> pgA, pgB;
  // autotuner
  bool tuned = false;
  bool snode_possible = false;
  std::string tune_path;
  std::string tune_key;
  int32_t* h_active = nullptr;
  int32_t* h_status = nullptr;
  int32_t* h_iters = nullptr;
  double* h_maxdx = nullptr;
  double* h_tol = nullptr;
  std::vector<mase::SysMeta> hsys;
  // continuous batching: per-slot snapshot ids, retire / refill tables and
  // the stream position (3 n_snap + 1 ints); per-snapshot results of the
  // stream (iterations, outcome), grown on demand
  int32_t* st_slots = nullptr;
  int32_t* st_out = nullptr;
  int64_t st_out_cap = 0;
  int32_t* h_st_active = nullptr;  // [2][n_snap] pinned: active flags of alternate passes
  int32_t* h_st_pos = nullptr;     // [2][2] pinned: stream position, lowest position in a slot
  int32_t* h_st_active_dev = nullptr;  // the same two buffers as the device addresses them
  int32_t* h_st_pos_dev = nullptr;
  hipEvent_t st_ev[2] = {};
  // device address, on this context's GPU, of the library's fixed scratch
  // array that mase_solve_stream_noalloc uses for the same bookkeeping
  int32_t* noalloc_scratch = nullptr;
  // per-stage timing
  bool prof = false;
  hipEvent_t pev[2 * MASE_N_STAGE] = {};
  bool pused[MASE_N_STAGE] = {};
  double pms[MASE_N_STAGE] = {};
  int64_t plaunch[MASE_N_STAGE] = {};
  int64_t punits[MASE_N_STAGE] = {};
};

namespace mase {
// Records msg as the thread's last error and returns code.
int set_error(int code, const std::string& msg);
// Launch of the batched objective (J per area and snapshot into jpart) at
// the state x (device, [n_snap][n_bus]).
int objective_at(mase_ctx* c, double2* x, double* jpart);
}  // namespace mase
