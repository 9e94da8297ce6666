// Host-side launch wrappers of the kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "dev.hpp"

namespace mase {

// LDS bytes of k_assemble for an area with nn local buses and nbr branches;
// br_lds: branch records staged in LDS too; nrow > 0: also the weights and
// measurements of the area's nrow rows.
size_t assemble_lds_bytes(int nn, int nbr, bool br_lds, int nrow);
hipError_t launch_assemble(const Dev& d, int a0, int na, int s0, int ns, int mode, size_t lds,
                           bool br_lds, hipStream_t st);
// lds: dynamic LDS bytes for the level staging (max over the launched systems)
hipError_t launch_eliminate(const Dev& d, int sys0, int nsys, int s0, int ns, size_t lds, hipStream_t st);
hipError_t allow_eliminate_lds(size_t bytes);
// the elimination with the area held in LDS, for the areas at positions
// [a0, a0 + na) of area_order: lds bytes (the largest of them), nt threads
// (256, 512 or 1024), tail_hbm if any of them keeps its Schur block in HBM
hipError_t launch_elim_lds(const Dev& d, int a0, int na, int s0, int ns, size_t lds, int nt, bool tail_hbm,
                           hipStream_t st);
// the back substitution of the same areas with their factor read into LDS
hipError_t launch_back_lds(const Dev& d, int a0, int na, int s0, int ns, size_t lds, int nt, bool fixed_bnd,
                           hipStream_t st);
hipError_t allow_elim_lds(size_t bytes);  // both kernels
// supernodal elimination of the boundary system's leading buses; lds: the
// plan's sn_lds_bytes
// supernodal elimination of the boundary system's leading buses (one
// workgroup per snapshot and subtree group), then their tail updates
hipError_t launch_gamma_snode(const Dev& d, int s0, int ns, size_t lds, hipStream_t st);
// back substitution of the same buses, supernode by supernode (after the dense block)
hipError_t launch_gamma_snode_back(const Dev& d, int s0, int ns, size_t lds, hipStream_t st);
hipError_t allow_gamma_snode_back_lds(size_t bytes);
hipError_t allow_gamma_snode_lds(size_t bytes);
hipError_t launch_gamma_gather(const Dev& d, int s0, int ns, int nslot, int nn, hipStream_t st);
// variants of the dense block's factorisation: 16-column steps on the matrix
// in HBM, the same with each 16-column panel staged in LDS, or nb-column
// panels staged whole in LDS (nb a multiple of 16, at most 64)
enum { DENSE_GLOBAL = 0, DENSE_PANEL16 = 1, DENSE_WIDE = 2 };
size_t dense_lds_bytes(int ld, int mode, int nb);
hipError_t launch_dense_chol(const Dev& d, int s0, int ns, int ld, int mode, int nb, hipStream_t st);
hipError_t allow_dense_lds(int mode, size_t bytes);
// fixed_bnd (areas): dx_b = 0 instead of E_k dx_Gamma (a local step, Eq. 6)
hipError_t launch_backsolve(const Dev& d, int sys0, int nsys, int s0, int ns, hipStream_t st,
                            bool fixed_bnd = false);
// local: boundary buses hold, convergence state untouched (a local step)
hipError_t launch_update(const Dev& d, int s0, int ns, hipStream_t st, bool local = false);
hipError_t launch_pack_state(const Dev& d, const double* vm, const double* va, double2* xout,
                             hipStream_t st);
hipError_t launch_unpack_state(const Dev& d, double* vm, double* va, hipStream_t st);
hipError_t launch_reset_flags(const Dev& d, hipStream_t st);
// continuous batching (one refill workgroup, then the slots' copies)
hipError_t launch_stream_refill(const Dev& d, int32_t* slot_id, int32_t* next, int32_t* retire,
                                int32_t* refill, int32_t* out_iters, int32_t* out_flag, int32_t n_total,
                                int32_t max_iter, int32_t* host_active, int32_t* host_pos, hipStream_t st);
hipError_t launch_stream_init(int32_t* slot_id, int32_t* next, int n_snap, hipStream_t st);
hipError_t launch_stream_copy(const Dev& d, const int32_t* retire, const int32_t* refill, const double* zs,
                              const double* vm0, const double* va0, double* vm_out, double* va_out,
                              hipStream_t st);
hipError_t allow_assemble_lds(size_t bytes, bool br_lds);

}  // namespace mase
