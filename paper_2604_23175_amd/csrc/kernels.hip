// HIP kernels of one Gauss-Newton iteration of multi-area WLS state
// estimation for gfx950 (arXiv 2604.23175, Sections 3-4).
//
//   k_assemble     fused measurement evaluation + accumulation of each area's
//                  G^k = H^T W H and b^k = H^T W r (Eq. 4, Eq. 7, Section 4.2)
//   k_eliminate    level-scheduled sparse Cholesky of the leading block with
//                  right-looking updates into the dense trailing block
//                  (Eq. 8-10, Section 4.3); also the sparse part of the
//                  boundary solve
//   k_gamma_gather boundary assembly S_Gamma = sum E_k^T S_b^k E_k (Eq. 11,
//                  Section 4.4), as a gather (no atomics)
//   k_gamma_snode  supernodal elimination of the boundary system's leading
//                  buses, independent elimination subtrees in parallel
//                  workgroups (FP64 MFMA panels); k_gamma_tail applies their
//                  updates of the dense block; k_gamma_snode_back is the
//                  matching back substitution
//   k_dense_wide   Cholesky + solve of the boundary system's dense block with
//                  64-column LDS panels (k_dense_chol: 16-column panels);
//                  trailing updates on FP64 MFMA
//   k_backsolve    scatter-back dx_b^k = E_k dx_Gamma and interior recovery
//                  dx_i^k = G_ii^-1 (b_i - G_ib dx_b) (Eq. 8)
//   k_update       x += dx, max |dx| per snapshot, convergence flags
//   k_stream_refill, k_stream_copy
//                  continuous batching: a slot whose snapshot has finished
//                  hands its result over and takes the next snapshot
//
// Every reduction has a fixed order, so results are bitwise reproducible.
// All arithmetic is FP64.
#include "dev.hpp"
#include "launch.hpp"

namespace mase {

namespace {

constexpr int VM = 0, QINJ = 2, PT = 5, QF = 4, QT = 6;
constexpr int ROLE_SELF = 0xFFFF;
constexpr int UP_SINGLE_FLAG = 1 << 30;  // update target with one inline contribution

// Workgroups are handed to the 8 XCDs round-robin by block index.  When the
// area count is a multiple of 8, all snapshots of one area land on one XCD so
// that the area's templates are shared through that XCD's L2.
__device__ inline void area_snap_of_block(int b, int na, int ns, int& ai, int& s) {
  if ((na & 7) == 0) {
    const int xcd = b & 7, slot = b >> 3;
    const int m = slot / ns;
    s = slot - m * ns;
    ai = xcd + 8 * m;
  } else {
    ai = b / ns;
    s = b - ai * ns;
  }
}

// Flow at end a of a branch (pi model): value and partials with respect to
// (theta_a, |V|_a) and (theta_o, |V|_o), where c, sn are cos and sin of
// theta_a - theta_o.  isq selects the reactive flow.
__device__ inline void flow_end(double g, double bs, double hb, double va, double vo, double c,
                                double sn, bool isq, double& h, double& dta, double& dva,
                                double& dto, double& dvo) {
  const double A = g * c + bs * sn;
  const double Bq = g * sn - bs * c;
  if (!isq) {
    h = g * va * va - va * vo * A;
    dta = va * vo * Bq;
    dva = 2.0 * g * va - vo * A;
    dvo = -va * A;
  } else {
    h = -(bs + hb) * va * va - va * vo * Bq;
    dta = -va * vo * A;
    dva = -2.0 * (bs + hb) * va - vo * Bq;
    dvo = -va * Bq;
  }
  dto = -dta;
}

// Branch record as staged in LDS.
struct BrL {
  double g, bs, hb;
  int lf, lt;
};

// Area-local evaluation context of the assembly kernel.
template <bool BR_LDS>
struct Asm {
  const Dev* d;
  int br0, slack_local;
  const double2* xs;   // local (theta, |V|)
  const double2* cs;   // cos, sin of theta_f - theta_t per local branch
  const double* agg;   // per local bus: P, Q, dP/dth, dP/dV, dQ/dth, dQ/dV
  const BrL* brl;      // branch records (BR_LDS)

  __device__ BrL branch(int e) const {
    if (BR_LDS) return brl[e];
    const int b = br0 + e;
    return BrL{d->br_g[b], d->br_bs[b], d->br_hb[b], d->br_lf[b], d->br_lt[b]};
  }

  // partials of the injection at bus u with respect to the bus across branch e
  __device__ int inj_nbr(int u, int e, bool q, double& dt, double& dv) const {
    const BrL B = branch(e);
    const bool from = (B.lf == u);
    const int o = from ? B.lt : B.lf;
    const double2 c = cs[e];
    double h, a1, a2;
    flow_end(B.g, B.bs, B.hb, xs[u].y, xs[o].y, c.x, from ? c.y : -c.y, q, h, a1, a2, dt, dv);
    return o;
  }

  // Value of the row rec = {type, loc, meas} and its partials with respect to
  // the buses picked by roles rp and rq.
  __device__ void eval2(int4 rec, int rp, int rq, double& h, double& pt, double& pv, double& qt,
                        double& qv) const {
    const int ty = rec.x, loc = rec.y;
    int bp, bq;
    if (ty == VM) {
      h = xs[loc].y;
      pt = qt = 0.0;
      pv = qv = 1.0;
      bp = bq = loc;
    } else if (ty <= QINJ) {
      const int q = (ty == QINJ) ? 1 : 0;
      const double* a = agg + 6 * loc;
      h = a[q];
      if (rp == ROLE_SELF) { pt = a[2 + 2 * q]; pv = a[3 + 2 * q]; bp = loc; }
      else bp = inj_nbr(loc, rp, q, pt, pv);
      if (rq == ROLE_SELF) { qt = a[2 + 2 * q]; qv = a[3 + 2 * q]; bq = loc; }
      else if (rq == rp) { qt = pt; qv = pv; bq = bp; }
      else bq = inj_nbr(loc, rq, q, qt, qv);
    } else {
      const BrL B = branch(loc);
      const bool to = (ty >= PT);
      const bool isq = (ty == QF || ty == QT);
      const int a = to ? B.lt : B.lf, o = to ? B.lf : B.lt;
      const double2 c = cs[loc];
      double ta, tv, to_, vo;
      flow_end(B.g, B.bs, B.hb, xs[a].y, xs[o].y, c.x, to ? -c.y : c.y, isq, h, ta, tv, to_, vo);
      if (rp == ROLE_SELF) { pt = ta; pv = tv; bp = a; } else { pt = to_; pv = vo; bp = o; }
      if (rq == ROLE_SELF) { qt = ta; qv = tv; bq = a; } else { qt = to_; qv = vo; bq = o; }
    }
    if (bp == slack_local) pt = 0.0;
    if (bq == slack_local) qt = 0.0;
  }

  // Partials, with respect to the bus across branch e from bus u, of the
  // active (dPt, dPv) and reactive (dQt, dQv) injections at u: those of
  // the two flows at u's end of e.  Returns that bus.
  __device__ int inj_nbr_pq(int u, int e, double& dPt, double& dPv, double& dQt, double& dQv) const {
    const BrL B = branch(e);
    const bool from = (B.lf == u);
    const int o = from ? B.lt : B.lf;
    const double2 c = cs[e];
    const double sn = from ? c.y : -c.y;
    const double va = xs[u].y, vo = xs[o].y;
    const double A = B.g * c.x + B.bs * sn;
    const double Bq = B.g * sn - B.bs * c.x;
    dPt = -(va * vo * Bq);
    dPv = -va * A;
    dQt = va * vo * A;
    dQv = -va * Bq;
    return o;
  }

  // One contribution record of a P/Q pair {family | loc << 3, meas P, meas Q,
  // roles}: values hP, hQ and the partials of both rows with respect to the
  // buses picked by roles rp (P: pt, pv; Q: qt... as Pp*, Qp*) and rq
  // (Pq*, Qq*).  Family VM: the P slot carries |V| (partials 0 and 1).
  __device__ void eval_pq(int fam, int loc, int rp, int rq, double& hP, double& hQ, double& Ppt,
                          double& Ppv, double& Pqt, double& Pqv, double& Qpt, double& Qpv, double& Qqt,
                          double& Qqv) const {
    int bp, bq;
    if (fam == VM) {
      hP = xs[loc].y;
      hQ = 0.0;
      Ppt = Pqt = Qpt = Qqt = 0.0;
      Ppv = Pqv = 1.0;
      Qpv = Qqv = 0.0;
      bp = bq = loc;
    } else if (fam < QINJ) {
      const double* a = agg + 6 * loc;
      hP = a[0];
      hQ = a[1];
      if (rp == ROLE_SELF) { Ppt = a[2]; Ppv = a[3]; Qpt = a[4]; Qpv = a[5]; bp = loc; }
      else bp = inj_nbr_pq(loc, rp, Ppt, Ppv, Qpt, Qpv);
      if (rq == ROLE_SELF) { Pqt = a[2]; Pqv = a[3]; Qqt = a[4]; Qqv = a[5]; bq = loc; }
      else if (rq == rp) { Pqt = Ppt; Pqv = Ppv; Qqt = Qpt; Qqv = Qpv; bq = bp; }
      else bq = inj_nbr_pq(loc, rq, Pqt, Pqv, Qqt, Qqv);
    } else {
      const BrL B = branch(loc);
      const bool to = (fam == PT);
      const int a = to ? B.lt : B.lf, o = to ? B.lf : B.lt;
      const double2 c = cs[loc];
      const double sn = to ? -c.y : c.y;
      const double va = xs[a].y, vo = xs[o].y;
      const double A = B.g * c.x + B.bs * sn;
      const double Bq = B.g * sn - B.bs * c.x;
      const double bsh = B.bs + B.hb;
      hP = B.g * va * va - va * vo * A;
      hQ = -bsh * va * va - va * vo * Bq;
      const double Pta = va * vo * Bq, Ptv = 2.0 * B.g * va - vo * A, Pov = -va * A;
      const double Qta = -va * vo * A, Qtv = -2.0 * bsh * va - vo * Bq, Qov = -va * Bq;
      if (rp == ROLE_SELF) { Ppt = Pta; Ppv = Ptv; Qpt = Qta; Qpv = Qtv; bp = a; }
      else { Ppt = -Pta; Ppv = Pov; Qpt = -Qta; Qpv = Qov; bp = o; }
      if (rq == ROLE_SELF) { Pqt = Pta; Pqv = Ptv; Qqt = Qta; Qqv = Qtv; bq = a; }
      else { Pqt = -Pta; Pqv = Pov; Qqt = -Qta; Qqv = Qov; bq = o; }
    }
    if (bp == slack_local) Ppt = Qpt = 0.0;
    if (bq == slack_local) Pqt = Qqt = 0.0;
  }
};

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  return t;
}

// Orders one wave's LDS writes before its following LDS reads across lanes.
// Lanes exchanging values through LDS is a data race in the language's model,
// so without this the compiler may, for instance, run the reading lanes of a
// divergent branch before the writing ones.
__device__ __attribute__((always_inline)) inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Plan records as plain structs (kept in registers across loops and
// barriers; the vector types' copy semantics can leave them on the stack).
struct alignas(16) Rec4 { int32_t x, y, z, w; };
struct alignas(8) Rec2 { int32_t x, y; };
__device__ inline Rec4 ld_rec(const int4* p) { return *reinterpret_cast<const Rec4*>(p); }
__device__ inline Rec2 ld_rec(const int2* p) { return *reinterpret_cast<const Rec2*>(p); }

// Workgroup barrier for threads that share data through LDS only: it waits
// for the wave's LDS operations but not for its global loads, so loads of
// read-only records issued before it stay in flight across it.  Global
// memory written by one thread and read by another is not ordered by it.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Value of v held by lane src (uniform across the wave) via the scalar unit.
__device__ inline double bcast_lane(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps.
__device__ inline double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * (1.5 - 0.5 * x * r * r);
  return r * (1.5 - 0.5 * x * r * r);
}

// Cholesky of the 16x16 diagonal block at (cb, cb) of the column-major LDS
// matrix P (pitch ldp) by one wave, with the forward solve of y[cb .. cb+15]
// and the inverse X = L^-1 built alongside.  The wave's lanes take three
// roles and run one instruction stream: lanes 0-15 hold row r = lane of the
// block (becoming row r of L), lanes 16-31 column j = lane - 16 of the
// identity (becoming column j of X), lane 32 the 16 entries of y.  At step c
// the pivot comes to all lanes through the scalar unit and 1/sqrt of it is the
// hardware estimate refined by two Newton steps; every lane scales its entry
// c by it (row lanes: L[r][c]; column lanes: X[c][j]; rhs lane: y_c) and then
// subtracts (its entry c) x L[m][c] from each entry m > c.  L[c+1][c], which
// the next pivot needs, comes through the scalar unit; the rest of column c
// through LDS: each lane writes its entry c to its own slot of a 64-double
// buffer (cxb: two of them, alternating, 128 doubles), so no store is
// divergent and no wave barrier splits the step -- one wave's LDS operations
// complete in order, and the compiler cannot move the read of slot m above
// the store to slot `lane`.  Every entry sees the same operations in the same
// order as a column-by-column right-looking factorisation.  Entries above the
// diagonal of a row lane pick up values that are never read or stored.  L
// goes back to P; Linv (row-major, pitch 17, zero above the diagonal)
// receives X, which turns the solves against L below the block into products
// on MFMA.  A non-positive pivot is reported by returning false; its column
// is then left unscaled (1/sqrt taken of 1 instead), and what follows is
// garbage for the caller to discard.
__device__ __attribute__((always_inline)) inline bool wave_chol16_inv4(double* P, int ldp, int cb, double* y,
                                                                       double* Linv, double* cxb) {
  const int lane = threadIdx.x & 63;
  int rr = lane & 15;
  asm volatile("" : "+v"(rr));  // per-lane predicates stay here, not hoisted into the caller
  const bool row = lane < 16, col = (lane >= 16 && lane < 32), rhs = lane == 32;
  double v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    double t = 0.0;
    if (row && m <= rr) t = P[(cb + m) * ldp + cb + rr];
    if (col && m == rr) t = 1.0;
    if (rhs) t = y[cb + m];
    v[m] = t;
  }
  // the start vector is formed here (else its loads sink into the loop and
  // stay live across it)
#pragma unroll
  for (int m = 0; m < 16; ++m) asm volatile("" : "+v"(v[m]));
  bool ok = true;
  double piv = bcast_lane(v[0], 0);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const bool good = piv > 0.0;
    ok = ok && good;
    const double inv = rsq_nr(good ? piv : 1.0);
    // row lane c holds the pivot itself, so this is pivot * 1/sqrt(pivot) there
    v[c] *= inv;
    if (c == 15) break;
    // a row lane above c multiplies garbage above its diagonal only
    const double f = v[c];
    double* cbuf = cxb + 64 * (c & 1);
    cbuf[lane] = v[c];
    v[c + 1] -= f * bcast_lane(v[c], c + 1);
    piv = bcast_lane(v[c + 1], c + 1);
#pragma unroll
    for (int m = c + 2; m < 16; ++m) v[m] -= f * cbuf[m];
    // this step's updates are applied now, not deferred to their next use
    // (which would keep every step's multipliers and LDS values live)
#pragma unroll
    for (int m = c + 2; m < 16; ++m) asm volatile("" : "+v"(v[m]));
  }
  if (row) {
#pragma unroll
    for (int m = 0; m < 16; ++m)
      if (m <= rr) P[(cb + m) * ldp + cb + rr] = v[m];
  }
  if (col) {
#pragma unroll
    for (int r = 0; r < 16; ++r) Linv[r * 17 + rr] = v[r];
  }
  if (rhs) {
#pragma unroll
    for (int r = 0; r < 16; ++r) y[cb + r] = v[r];
  }
  return ok;
}

__device__ inline double nanmax(double m, double v) { return (v > m || v != v) ? v : m; }

__device__ inline double block_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = nanmax(t, red[i]);
  return t;
}

// 2x2 Cholesky of [[a00, .], [a10, a11]] with the reciprocals i00 = 1/l00,
// i11 = 1/l11 (the solves multiply by them); false on a non-positive pivot.
__device__ inline bool chol2(double a00, double a10, double a11, double& l00, double& l10, double& l11,
                             double& i00, double& i11) {
  if (!(a00 > 0.0)) return false;
  i00 = rsq_nr(a00);
  l00 = a00 * i00;
  l10 = a10 * i00;
  const double p = a11 - l10 * l10;
  if (!(p > 0.0)) return false;
  i11 = rsq_nr(p);
  l11 = p * i11;
  return true;
}

__device__ inline bool chol2(double a00, double a10, double a11, double& l00, double& l10, double& l11) {
  double i00, i11;
  return chol2(a00, a10, a11, l00, l10, l11, i00, i11);
}

}  // namespace

// ---------------------------------------------------------------------------
// Stage 1: fused evaluation and accumulation (one workgroup per area x
// snapshot).  LDS holds the area's local states, cos/sin of every local
// branch's angle difference, every own bus's injection value and
// self-partials (sums over incident branch ends: Kirchhoff's current law) and,
// when it fits, the branch records.  G slots are visited in packed-storage
// order and each sums its precomputed, fixed-order contribution list, so the
// writes are contiguous and the sum is deterministic.
// ---------------------------------------------------------------------------
// 16 waves per workgroup: the area's LDS staging limits a CU to one or two
// workgroups, and the gathers are latency-bound, so waves are what hide it.
constexpr int ASM_NT = 1024;

// WZ: the rows' weights and measurements are staged in LDS (with the area).
template <bool BR_LDS, bool STAGE_HBM, bool WZ>
__global__ void __launch_bounds__(ASM_NT) k_assemble(Dev d, int a0, int na, int s0, int ns, int mode) {
  static_assert(!(WZ && STAGE_HBM), "weights are staged only with the area in LDS");
  int ai, s;
  area_snap_of_block(blockIdx.x, na, ns, ai, s);
  s += s0;
  const int k = d.area_order[a0 + ai];
  if (mode == MODE_ASSEMBLE && !d.active[s]) return;
  const AreaMeta am = d.area[k];
  const SysMeta sm = d.sys[k];
  extern __shared__ double2 lds2[];
  __shared__ double red[16];
  // staging: LDS, or (areas too large for it) this block's region of HBM
  double2* xs = STAGE_HBM ? reinterpret_cast<double2*>(d.asm_stage + (int64_t)s * d.asm_stride + am.stage_off)
                          : lds2;
  double2* cs = xs + am.nn;
  double* agg = reinterpret_cast<double*>(cs + am.nbr);
  BrL* brl = reinterpret_cast<BrL*>(agg + 6 * am.nn);
  // weight and measurement of every row of the area (assembly with staging in LDS)
  double2* wzs = reinterpret_cast<double2*>(brl + (BR_LDS ? am.nbr : 0));
  const double2* xsnap = d.x + (int64_t)s * d.n_bus;
  const int tid = threadIdx.x, nt = blockDim.x;

  for (int v = tid; v < am.nn; v += nt) xs[v] = xsnap[d.gbus[sm.gbus + v]];
  if (WZ && mode == MODE_ASSEMBLE) {
    const double* zsn = d.z + (int64_t)s * d.n_meas;
    for (int r = tid; r < am.nrow; r += nt) {
      const int m = d.rowrec[am.row + r].z;
      wzs[r] = make_double2(d.w[m], zsn[m]);
    }
  }
  if (BR_LDS)
    for (int e = tid; e < am.nbr; e += nt) {
      const int b = am.br + e;
      brl[e] = BrL{d.br_g[b], d.br_bs[b], d.br_hb[b], d.br_lf[b], d.br_lt[b]};
    }
  __syncthreads();
  const Asm<BR_LDS> X{&d, am.br, am.slack_local, xs, cs, agg, brl};
  for (int e = tid; e < am.nbr; e += nt) {
    const BrL B = X.branch(e);
    double sn, c;
    sincos(xs[B.lf].x - xs[B.lt].x, &sn, &c);
    cs[e] = make_double2(c, sn);
  }
  __syncthreads();
  for (int v = tid; v < am.nn; v += nt) {
    const int p0 = d.inc_ptr[am.inc_ptr + v], p1 = d.inc_ptr[am.inc_ptr + v + 1];
    double P = 0, Q = 0, dPt = 0, dPv = 0, dQt = 0, dQv = 0;
    for (int q = p0; q < p1; ++q) {
      const int code = d.inc_end[q];
      const int le = code >> 1, side = code & 1;
      const BrL B = X.branch(le);
      const int o = side ? B.lf : B.lt;
      const double2 c = cs[le];
      const double sn = side ? -c.y : c.y;
      double h, ta, tv, to_, vo;
      flow_end(B.g, B.bs, B.hb, xs[v].y, xs[o].y, c.x, sn, false, h, ta, tv, to_, vo);
      P += h; dPt += ta; dPv += tv;
      flow_end(B.g, B.bs, B.hb, xs[v].y, xs[o].y, c.x, sn, true, h, ta, tv, to_, vo);
      Q += h; dQt += ta; dQv += tv;
    }
    double* a = agg + 6 * v;
    a[0] = P; a[1] = Q; a[2] = dPt; a[3] = dPv; a[4] = dQt; a[5] = dQv;
  }
  __syncthreads();

  const double* zs = d.z + (int64_t)s * d.n_meas;
  if (mode == MODE_EVAL_H) {
    for (int r = tid; r < am.nrow; r += nt) {
      const int4 rec = d.rowrec[am.row + r];
      double h, a1, a2, a3, a4;
      X.eval2(rec, ROLE_SELF, ROLE_SELF, h, a1, a2, a3, a4);
      d.hout[(int64_t)s * d.n_meas + rec.z] = h;
    }
    return;
  }
  // objective J = sum w r^2 over the area's rows (Eq. 2), objective mode only
  if (mode == MODE_OBJECTIVE) {
    double jl = 0.0;
    for (int r = tid; r < am.nrow; r += nt) {
      const int4 rec = d.rowrec[am.row + r];
      double h, a1, a2, a3, a4;
      X.eval2(rec, ROLE_SELF, ROLE_SELF, h, a1, a2, a3, a4);
      const double res = zs[rec.z] - h;
      jl += d.w[rec.z] * res * res;
    }
    const double jt = block_sum(jl, red);
    if (tid == 0) d.jpart[(int64_t)s * d.n_area + k] = jt;
    return;
  }

  // G^k slots: slot += w * h_p h_q^T over the slot's contributions.  The
  // diagonal slot (v, v) also sums b_v = sum w r h_v (Eq. 7) over its
  // contributions with equal roles, which are exactly bus v's rows.
  double* vals = d.vals + (int64_t)s * d.vstride + sm.val_off;
  double* rhs = d.rhs + (int64_t)s * d.rstride + sm.rhs_off;
  // Each record is a P/Q pair of rows (or a single row): its two rows share
  // the branch terms, so both are evaluated at once.  A wave's 64 lanes
  // handle 64 consecutive slots, whose c-th records lie side by side (one
  // coalesced load per step); the weights and measurements of the area's
  // rows are staged in LDS (wz) when they fit.  The next record is in flight
  // while one is evaluated, and the next slot's header and first record are
  // requested before this slot's results are stored.
  auto wz_of = [&](int r) -> double2 {
    if constexpr (WZ) {
      return wzs[r];
    } else {
      const int m = d.rowrec[am.row + r].z;
      return make_double2(d.w[m], zs[m]);
    }
  };
  const int lane = tid & 63;
  const int4 zero4 = make_int4(0, -1, -1, 0);
  int i = tid;
  int4 sl = i < am.nslot ? d.slot[am.slot + i] : zero4;
  int rb2 = i < am.nslot ? d.slot_rhs[am.slot + i] : -1;
  // Two records in flight.  A slot's contribution records are taken
  // alternately from two registers, each refilled (unconditionally, the index
  // clamped to the slot's last record) as soon as its record has been taken,
  // so that the loads stay in flight across the contributions' arithmetic
  // (a wave's loads complete in issue order, and a conditional load would
  // make every later wait cover all of them).
  double c00 = 0, c10 = 0, c01 = 0, c11 = 0, b0 = 0, b1 = 0;
  auto contribution = [&](const int4 cr) {
    const int rp = cr.w & 0xFFFF, rq = (cr.w >> 16) & 0xFFFF;
    double hP, hQ, Ppt, Ppv, Pqt, Pqv, Qpt, Qpv, Qqt, Qqv;
    X.eval_pq(cr.x & 7, cr.x >> 3, rp, rq, hP, hQ, Ppt, Ppv, Pqt, Pqv, Qpt, Qpv, Qqt, Qqv);
    if (cr.y >= 0) {
      const double2 wzp = wz_of(cr.y);
      if (rb2 >= 0 && rp == rq) {
        const double wres = wzp.x * (wzp.y - hP);
        b0 += Ppt * wres;
        b1 += Ppv * wres;
      }
      Ppt *= wzp.x;
      Ppv *= wzp.x;
      c00 += Ppt * Pqt;
      c10 += Ppv * Pqt;
      c01 += Ppt * Pqv;
      c11 += Ppv * Pqv;
    }
    if (cr.z >= 0) {
      const double2 wzq = wz_of(cr.z);
      if (rb2 >= 0 && rp == rq) {
        const double wres = wzq.x * (wzq.y - hQ);
        b0 += Qpt * wres;
        b1 += Qpv * wres;
      }
      Qpt *= wzq.x;
      Qpv *= wzq.x;
      c00 += Qpt * Qqt;
      c10 += Qpv * Qqt;
      c01 += Qpt * Qqv;
      c11 += Qpv * Qqv;
    }
  };
  int4 rA = d.scon[(i < am.nslot && sl.w > 0) ? sl.z + lane : 0];
  int4 rB = d.scon[(i < am.nslot && sl.w > 1) ? sl.z + 64 + lane : 0];
  for (; i < am.nslot; i += nt) {
    c00 = c10 = c01 = c11 = b0 = b1 = 0;
    const int w = sl.w;
    for (int c = 0; c < w; c += 2) {
      const int4 ca = rA;
      rA = d.scon[sl.z + min(c + 2, w - 1) * 64 + lane];
      contribution(ca);
      const int4 cb = rB;
      rB = d.scon[sl.z + min(c + 3, w - 1) * 64 + lane];
      if (c + 1 < w) contribution(cb);
    }
    // the next slot, requested before the stores below
    const int in = i + nt;
    const int inc = in < am.nslot ? in : am.nslot - 1;
    const int4 slr = d.slot[am.slot + inc];
    const int rbr = d.slot_rhs[am.slot + inc];
    const int4 sln = in < am.nslot ? slr : zero4;
    const int rbn = in < am.nslot ? rbr : -1;
    rA = d.scon[(in < am.nslot && sln.w > 0) ? sln.z + lane : 0];
    rB = d.scon[(in < am.nslot && sln.w > 1) ? sln.z + 64 + lane : 0];
    const bool diag = sl.y < 0;
    const int stride = diag ? -sl.y : sl.y;
    if (diag) c01 = c10;
    if (sl.x == sm.asm_pin) { c00 = 1.0; c10 = 0.0; c01 = 0.0; }
    double* o = vals + sl.x;
    o[0] = c00;
    o[1] = c10;
    o[stride] = c01;
    o[stride + 1] = c11;
    if (rb2 >= 0) {
      rhs[rb2] = b0;
      rhs[rb2 + 1] = b1;
    }
    sl = sln;
    rb2 = rbn;
  }
}

// ---------------------------------------------------------------------------
// Stage 2 (and the sparse part of stage 3): level-scheduled elimination of a
// system's leading buses.  One workgroup per system x snapshot.  For each
// elimination-tree level: (a) every column of the level divides by its 2x2
// pivot (recomputed from the stored, fully updated diagonal block, which is
// never overwritten) and forms y_j = L_jj^-1 b_j; (b) every update target of
// the level (a 2x2 block in a later column or in the dense tail) subtracts
// sum_j L_ij L_pj^T in a fixed order, and every rhs target subtracts
// sum_j L_ij y_j.  After the last level the tail holds the Schur complement
// S_b = G_bb - G_bi G_ii^-1 G_ib and the tail rhs holds bhat_b (Eq. 9-10).
// ---------------------------------------------------------------------------
template <int NT, bool RL>
__global__ void __launch_bounds__(NT) k_eliminate(Dev d, int sys0, int nsys, int s0, int ns, int lstride) {
  int si, s;
  area_snap_of_block(blockIdx.x, nsys, ns, si, s);
  s += s0;
  if (!d.active[s]) return;
  const int k = (sys0 < d.n_area) ? d.area_order[sys0 + si] : sys0 + si;
  const SysMeta sm = d.sys[k];
  double* vals = d.vals + (int64_t)s * d.vstride + sm.val_off;
  double* rhs_g = d.rhs + (int64_t)s * d.rstride + sm.rhs_off;
  // the level's new factor blocks (4 doubles each) and y_j (2 each); after
  // them (lstride doubles in) the system's rhs, kept in LDS throughout when
  // the largest system's fits (RL)
  extern __shared__ double2 lstage2[];
  double* lst = reinterpret_cast<double*>(lstage2);
  double* rhs = RL ? lst + lstride : rhs_g;
  const int tid = threadIdx.x;
  if (RL) {
    for (int i = tid; i < 2 * sm.nn; i += NT) rhs[i] = rhs_g[i];
    __syncthreads();
  }
  bool bad = false;
  // Latency structure.  A wave's loads complete in issue order (one counter
  // for loads and stores), so a record fetched early but consumed after a
  // later load costs nothing only if nothing waits in between.  Each level
  // therefore issues, in one burst, every load of its first pass (the pivot
  // and column blocks of its first column item, the current values of its
  // first UB update targets with their first contribution records, the
  // first contribution of its first rhs target) together with the next
  // level's first records and the level bounds two levels ahead; one wait
  // covers them all.  Update targets of a level lie in later columns, which
  // the level's column phase does not write, so their values can be read
  // before it, and the barrier between the phases only orders LDS.  The
  // barrier that closes a level waits for its stores, which the next level
  // reads.  Items beyond the first pass load their records and values on
  // demand.  Every value sees the same operations in the same order as a
  // plain level-by-level schedule.
  constexpr int UB = 2;
  const int32_t* cdp = d.cd_ptr + sm.cd_ptr;
  const int32_t* upp = d.up_ptr + sm.up_ptr;
  const int32_t* rbp = d.rb_ptr + sm.rb_ptr;
  const int nlev = sm.nlev;
  const Rec4 none{-1, 0, 0, 0};
  // bounds of this level [c0, c1) ... and the next level's ends nc1, nu1, nr1
  int c0 = 0, c1 = 0, u0 = 0, u1 = 0, r0 = 0, r1 = 0, nc1 = 0, nu1 = 0, nr1 = 0;
  Rec4 crec = none, rrec = none;
  Rec4 trec[UB];
#pragma unroll
  for (int q = 0; q < UB; ++q) trec[q] = none;
  if (nlev > 0) {
    c0 = __builtin_amdgcn_readfirstlane(cdp[0]);
    c1 = __builtin_amdgcn_readfirstlane(cdp[1]);
    u0 = __builtin_amdgcn_readfirstlane(upp[0]);
    u1 = __builtin_amdgcn_readfirstlane(upp[1]);
    r0 = __builtin_amdgcn_readfirstlane(rbp[0]);
    r1 = __builtin_amdgcn_readfirstlane(rbp[1]);
    nc1 = __builtin_amdgcn_readfirstlane(nlev > 1 ? cdp[2] : c1);
    nu1 = __builtin_amdgcn_readfirstlane(nlev > 1 ? upp[2] : u1);
    nr1 = __builtin_amdgcn_readfirstlane(nlev > 1 ? rbp[2] : r1);
    if (c0 + tid < c1) crec = ld_rec(d.cd_items + c0 + tid);
#pragma unroll
    for (int q = 0; q < UB; ++q)
      if (u0 + tid + q * NT < u1) trec[q] = ld_rec(d.up_tgt + u0 + tid + q * NT);
    if (r0 + tid < r1) rrec = ld_rec(d.rb_tgt + r0 + tid);
  }
  for (int lev = 0; lev < nlev; ++lev) {
    // ---- the burst: this level's first-pass values and contribution records
    double dv0 = 0, dv1 = 0, dv3 = 0;
    double2 mv0 = make_double2(0, 0), mv1 = make_double2(0, 0);
    if (crec.x >= 0) {
      const double* D = vals + crec.x;
      dv0 = D[0];
      dv1 = D[1];
      dv3 = D[3];
      if (crec.y >= 0) {
        const double* M = vals + crec.y;
        mv0 = *reinterpret_cast<const double2*>(M);
        mv1 = *reinterpret_cast<const double2*>(M + 2);
      }
    }
    double cv[UB][4];
    Rec2 uc[UB];
#pragma unroll
    for (int q = 0; q < UB; ++q) {
      uc[q] = Rec2{0, 0};
      cv[q][0] = cv[q][1] = cv[q][2] = cv[q][3] = 0.0;
      if (trec[q].x >= 0) {
        const int stride = trec[q].y & ~UP_SINGLE_FLAG;
        const double* C = vals + trec[q].x;
        cv[q][0] = C[0];
        cv[q][1] = C[1];
        cv[q][2] = C[stride];
        cv[q][3] = C[stride + 1];
        if (!(trec[q].y & UP_SINGLE_FLAG)) uc[q] = ld_rec(d.up_con + trec[q].z);
      }
    }
    Rec2 rc{0, 0};
    if (rrec.x >= 0 && rrec.y < rrec.z) rc = ld_rec(d.rb_con + rrec.y);
    // ---- the next level's first records and the bounds after it
    const bool more = lev + 1 < nlev;
    Rec4 cn = none, rn = none;
    Rec4 tn[UB];
#pragma unroll
    for (int q = 0; q < UB; ++q) tn[q] = none;
    int nnc1 = nc1, nnu1 = nu1, nnr1 = nr1;
    if (more) {
      if (c1 + tid < nc1) cn = ld_rec(d.cd_items + c1 + tid);
#pragma unroll
      for (int q = 0; q < UB; ++q)
        if (u1 + tid + q * NT < nu1) tn[q] = ld_rec(d.up_tgt + u1 + tid + q * NT);
      if (r1 + tid < nr1) rn = ld_rec(d.rb_tgt + r1 + tid);
      if (lev + 2 < nlev) {
        nnc1 = cdp[lev + 3];
        nnu1 = upp[lev + 3];
        nnr1 = rbp[lev + 3];
      }
    }
    // every wave waits for the burst here, so no later use of its data
    // waits behind the stores this level issues
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // ---- column phase: pivots, y_j, and the column blocks X with X L^T = M
    for (int it = c0 + tid; it < c1; it += NT) {
      const bool first = it == c0 + tid;
      const Rec4 c = first ? crec : ld_rec(d.cd_items + it);
      double a00, a10, a11;
      if (first) {
        a00 = dv0; a10 = dv1; a11 = dv3;
      } else {
        const double* D = vals + c.x;
        a00 = D[0]; a10 = D[1]; a11 = D[3];
      }
      double l00, l10, l11, i00, i11;
      if (!chol2(a00, a10, a11, l00, l10, l11, i00, i11)) {
        bad = true;
        l00 = l11 = i00 = i11 = 1.0;
        l10 = 0.0;
      }
      if (c.y < 0) {
        const double y0 = rhs[c.z] * i00;
        const double y1 = (rhs[c.z + 1] - l10 * y0) * i11;
        rhs[c.z] = y0;
        rhs[c.z + 1] = y1;
        lst[c.w] = y0;
        lst[c.w + 1] = y1;
      } else {
        double* M = vals + c.y;
        double2 m0, m1;
        if (first) {
          m0 = mv0; m1 = mv1;
        } else {
          m0 = *reinterpret_cast<const double2*>(M);
          m1 = *reinterpret_cast<const double2*>(M + 2);
        }
        const double x00 = m0.x * i00, x10 = m0.y * i00;
        const double x01 = (m1.x - x00 * l10) * i11, x11 = (m1.y - x10 * l10) * i11;
        *reinterpret_cast<double2*>(M) = make_double2(x00, x10);
        *reinterpret_cast<double2*>(M + 2) = make_double2(x01, x11);
        *reinterpret_cast<double2*>(lst + c.w) = make_double2(x00, x10);
        *reinterpret_cast<double2*>(lst + c.w + 2) = make_double2(x01, x11);
      }
    }
    // the update phase reads the column phase's results from LDS only
    // (with the rhs in HBM, y_i of a later column is not written above)
    lds_barrier();
    // ---- update phase: target -= sum_j L_ij L_pj^T, fixed order
    auto update = [&](const Rec4 t, double c00, double c10, double c01, double c11, Rec2 p0) {
      double a00 = 0, a10 = 0, a01 = 0, a11 = 0;
      const bool single = (t.y & UP_SINGLE_FLAG) != 0;
      const int stride = t.y & ~UP_SINGLE_FLAG;
      auto acc = [&](const Rec2 u) {
        const double2 L0 = *reinterpret_cast<const double2*>(lst + u.x);
        const double2 L1 = *reinterpret_cast<const double2*>(lst + u.x + 2);
        const double2 P0 = *reinterpret_cast<const double2*>(lst + u.y);
        const double2 P1 = *reinterpret_cast<const double2*>(lst + u.y + 2);
        a00 += L0.x * P0.x + L1.x * P1.x;
        a10 += L0.y * P0.x + L1.y * P1.x;
        a01 += L0.x * P0.y + L1.x * P1.y;
        a11 += L0.y * P0.y + L1.y * P1.y;
      };
      // the first contribution is in registers already (no wait behind this
      // level's stores); further ones are loaded here
      Rec2 u = single ? Rec2{t.z, t.w} : p0;
      acc(u);
      if (!single)
        for (int c = t.z + 1; c < t.w; ++c) {
          u = ld_rec(d.up_con + c);
          acc(u);
        }
      if (u.x == u.y) a01 = a10;
      double* C = vals + t.x;
      C[0] = c00 - a00;
      C[1] = c10 - a10;
      C[stride] = c01 - a01;
      C[stride + 1] = c11 - a11;
    };
#pragma unroll
    for (int q = 0; q < UB; ++q)
      if (trec[q].x >= 0) update(trec[q], cv[q][0], cv[q][1], cv[q][2], cv[q][3], uc[q]);
    for (int it0 = u0 + tid + NT * UB; it0 < u1; it0 += NT * UB) {
      Rec4 t[UB];
      double c00[UB], c10[UB], c01[UB], c11[UB];
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        const int it = it0 + q * NT;
        t[q] = it < u1 ? ld_rec(d.up_tgt + it) : none;
      }
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        if (t[q].x < 0) continue;
        const int stride = t[q].y & ~UP_SINGLE_FLAG;
        const double* C = vals + t[q].x;
        c00[q] = C[0];
        c10[q] = C[1];
        c01[q] = C[stride];
        c11[q] = C[stride + 1];
      }
#pragma unroll
      for (int q = 0; q < UB; ++q) {
        if (t[q].x < 0) continue;
        const bool single = (t[q].y & UP_SINGLE_FLAG) != 0;
        const Rec2 p0 = single ? Rec2{0, 0} : ld_rec(d.up_con + t[q].z);
        update(t[q], c00[q], c10[q], c01[q], c11[q], p0);
      }
    }
    // ---- rhs targets: y_i -= sum_j L_ij y_j
    for (int it = r0 + tid; it < r1; it += NT) {
      const bool first = it == r0 + tid;
      const Rec4 t = first ? rrec : ld_rec(d.rb_tgt + it);
      double b0 = 0, b1 = 0;
      auto acc = [&](const Rec2 u) {
        const double* L = lst + u.x;
        const double y0 = lst[u.y], y1 = lst[u.y + 1];
        b0 += L[0] * y0 + L[2] * y1;
        b1 += L[1] * y0 + L[3] * y1;
      };
      if (t.y < t.z) acc(first ? rc : ld_rec(d.rb_con + t.y));
      for (int c = t.y + 1; c < t.z; ++c) acc(ld_rec(d.rb_con + c));
      rhs[t.x] -= b0;
      rhs[t.x + 1] -= b1;
    }
    // the next level reads the blocks stored above
    __syncthreads();
    // level bounds are uniform: keep them in scalar registers
    c0 = c1; c1 = nc1; u0 = u1; u1 = nu1; r0 = r1; r1 = nr1;
    nc1 = __builtin_amdgcn_readfirstlane(nnc1);
    nu1 = __builtin_amdgcn_readfirstlane(nnu1);
    nr1 = __builtin_amdgcn_readfirstlane(nnr1);
    crec = cn;
    rrec = rn;
#pragma unroll
    for (int q = 0; q < UB; ++q) trec[q] = tn[q];
  }
  if (RL)
    for (int i = tid; i < 2 * sm.nn; i += NT) rhs_g[i] = rhs[i];
  if (bad) d.status[(int64_t)s * (d.n_area + 1) + k] = 1;
}

// ---------------------------------------------------------------------------
// Stage 2 with the area held in LDS.  One workgroup per area x snapshot
// keeps the area's packed storage [0, split) and its rhs in LDS for the whole
// elimination: it zeroes the image, drops in the compact G blocks the
// assembly wrote (fill positions stay zero), runs the same level schedule as
// k_eliminate with every factor block, pivot and update in LDS, and writes the
// storage back once (the factor for the back substitution, S_b^k for the
// boundary assembly).  HBM sees G read once and L written once instead of a
// read-modify-write round trip per level.  With TAIL_HBM the area does not
// fit whole: its Schur block [split, nval) stays in HBM, already assembled
// there, and only the updates that land in it go to HBM.  The arithmetic and
// its order are those of k_eliminate, so results are bitwise the same.
// ---------------------------------------------------------------------------
template <int NT, bool TAIL_HBM>
__global__ void __launch_bounds__(NT) k_elim_lds(Dev d, int a0, int na, int s0, int ns) {
  int ai, s;
  area_snap_of_block(blockIdx.x, na, ns, ai, s);
  s += s0;
  if (!d.active[s]) return;
  const int k = d.area_order[a0 + ai];
  const SysMeta sm = d.sys[k];
  const AreaMeta am = d.area[k];
  double* vals = d.vals + (int64_t)s * d.vstride + sm.val_off;
  double* rhs_g = d.rhs + (int64_t)s * d.rstride + sm.rhs_off;
  extern __shared__ double2 lds2[];
  double* img = reinterpret_cast<double*>(lds2);
  const int split = am.split;  // a multiple of 4
  double* rhs = img + split;
  const int tid = threadIdx.x;
  for (int i = tid; i < split / 2; i += NT) lds2[i] = make_double2(0.0, 0.0);
  for (int i = tid; i < sm.nn; i += NT)
    reinterpret_cast<double2*>(rhs)[i] = reinterpret_cast<const double2*>(rhs_g)[i];
  __syncthreads();
  {
    const double2* gc = reinterpret_cast<const double2*>(vals + am.gc_rel);
    const int32_t* cimg = d.cimg + am.cimg;
    for (int i = tid; i < am.n_cslot; i += NT) {
      const double2 lo = gc[2 * i], hi = gc[2 * i + 1];
      double2* dst = reinterpret_cast<double2*>(img + cimg[i]);
      dst[0] = lo;
      dst[1] = hi;
    }
  }
  __syncthreads();
  bool bad = false;
  const int32_t* cdp = d.cd_ptr + sm.cd_ptr;
  const int32_t* upp = d.up_ptr + sm.up_ptr;
  const int32_t* rbp = d.rb_ptr + sm.rb_ptr;
  // Each level's first records per thread (its first column item, its first
  // two update targets, its first rhs target) are loaded one level ahead.
  // Threads share values through LDS only, so the barriers between phases
  // wait for LDS traffic alone and those loads stay in flight across them;
  // with the Schur block in HBM (TAIL_HBM) its read-modify-writes need the
  // full workgroup barrier.
  const Rec4 none{-1, 0, 0, 0};
  int c0 = 0, c1 = 0, u0 = 0, u1 = 0, r0 = 0, r1 = 0;
  Rec4 cpre = none, tpre0 = none, tpre1 = none, rpre = none;  // two update targets per pass
  if (sm.nlev > 0) {
    c0 = cdp[0]; c1 = cdp[1]; u0 = upp[0]; u1 = upp[1]; r0 = rbp[0]; r1 = rbp[1];
    if (c0 + tid < c1) cpre = ld_rec(d.cd_items + c0 + tid);
    if (u0 + tid < u1) tpre0 = ld_rec(d.up_tgt_img + u0 + tid);
    if (u0 + tid + NT < u1) tpre1 = ld_rec(d.up_tgt_img + u0 + tid + NT);
    if (r0 + tid < r1) rpre = ld_rec(d.rb_tgt + r0 + tid);
  }
  for (int lev = 0; lev < sm.nlev; ++lev) {
    const bool more = lev + 1 < sm.nlev;
    const int nc1 = more ? cdp[lev + 2] : c1, nu1 = more ? upp[lev + 2] : u1, nr1 = more ? rbp[lev + 2] : r1;
    // first contribution of this thread's first rhs target
    Rec2 rc{0, 0};
    if (r0 + tid < r1 && rpre.y < rpre.z) rc = ld_rec(d.rb_con_img + rpre.y);
    // the next level's records, in flight while this level runs
    Rec4 cnext = none, tnext0 = none, tnext1 = none, rnext = none;
    if (more && c1 + tid < nc1) cnext = ld_rec(d.cd_items + c1 + tid);
    if (more && u1 + tid < nu1) tnext0 = ld_rec(d.up_tgt_img + u1 + tid);
    if (more && u1 + tid + NT < nu1) tnext1 = ld_rec(d.up_tgt_img + u1 + tid + NT);
    if (more && r1 + tid < nr1) rnext = ld_rec(d.rb_tgt + r1 + tid);

    for (int it = c0 + tid; it < c1; it += NT) {
      const Rec4 c = (it == c0 + tid) ? cpre : ld_rec(d.cd_items + it);
      const double* D = img + c.x;
      double l00, l10, l11, i00, i11;
      if (!chol2(D[0], D[1], D[3], l00, l10, l11, i00, i11)) {
        bad = true;
        l00 = l11 = i00 = i11 = 1.0;
        l10 = 0.0;
      }
      if (c.y < 0) {
        const double y0 = rhs[c.z] * i00;
        const double y1 = (rhs[c.z + 1] - l10 * y0) * i11;
        rhs[c.z] = y0;
        rhs[c.z + 1] = y1;
      } else {
        double2* M = reinterpret_cast<double2*>(img + c.y);  // X L^T = M
        const double2 m0 = M[0], m1 = M[1];
        const double x00 = m0.x * i00, x10 = m0.y * i00;
        const double x01 = (m1.x - x00 * l10) * i11, x11 = (m1.y - x10 * l10) * i11;
        M[0] = make_double2(x00, x10);
        M[1] = make_double2(x01, x11);
      }
    }
    if constexpr (TAIL_HBM) __syncthreads();
    else lds_barrier();
    auto update = [&](const Rec4 t) {
      const bool single = (t.y & UP_SINGLE_FLAG) != 0;
      const int stride = t.y & ~UP_SINGLE_FLAG;
      const int cb = single ? 0 : t.z, ce = single ? 1 : t.w;
      double a00 = 0, a10 = 0, a01 = 0, a11 = 0;
      bool sym = false;
      for (int c = cb; c < ce; ++c) {
        const Rec2 u = single ? Rec2{t.z, t.w} : ld_rec(d.up_con_img + c);
        const double2 L0 = *reinterpret_cast<const double2*>(img + u.x);
        const double2 L1 = *reinterpret_cast<const double2*>(img + u.x + 2);
        const double2 P0 = *reinterpret_cast<const double2*>(img + u.y);
        const double2 P1 = *reinterpret_cast<const double2*>(img + u.y + 2);
        a00 += L0.x * P0.x + L1.x * P1.x;
        a10 += L0.y * P0.x + L1.y * P1.x;
        a01 += L0.x * P0.y + L1.x * P1.y;
        a11 += L0.y * P0.y + L1.y * P1.y;
        sym = (u.x == u.y);
      }
      if (sym) a01 = a10;
      double* C = (!TAIL_HBM || t.x < split) ? img + t.x : vals + t.x;
      const double c00 = C[0], c10 = C[1], c01 = C[stride], c11 = C[stride + 1];
      C[0] = c00 - a00;
      C[1] = c10 - a10;
      C[stride] = c01 - a01;
      C[stride + 1] = c11 - a11;
    };
    for (int it0 = u0 + tid; it0 < u1; it0 += 2 * NT) {
      const bool first = it0 == u0 + tid;
      const Rec4 ta = first ? tpre0 : ld_rec(d.up_tgt_img + it0);
      const Rec4 tb = first ? tpre1 : (it0 + NT < u1 ? ld_rec(d.up_tgt_img + it0 + NT) : none);
      update(ta);
      if (tb.x >= 0) update(tb);
    }
    for (int it = r0 + tid; it < r1; it += NT) {
      const bool first = it == r0 + tid;
      const Rec4 t = first ? rpre : ld_rec(d.rb_tgt + it);
      double b0 = 0, b1 = 0;
      for (int c = t.y; c < t.z; ++c) {
        const Rec2 u = (first && c == t.y) ? rc : ld_rec(d.rb_con_img + c);
        const double* L = img + u.x;
        const double y0 = rhs[u.y], y1 = rhs[u.y + 1];
        b0 += L[0] * y0 + L[2] * y1;
        b1 += L[1] * y0 + L[3] * y1;
      }
      rhs[t.x] -= b0;
      rhs[t.x + 1] -= b1;
    }
    if constexpr (TAIL_HBM) __syncthreads();
    else lds_barrier();
    c0 = c1; c1 = nc1; u0 = u1; u1 = nu1; r0 = r1; r1 = nr1;
    cpre = cnext;
    tpre0 = tnext0;
    tpre1 = tnext1;
    rpre = rnext;
  }
  double2* v2 = reinterpret_cast<double2*>(vals);
  for (int i = tid; i < split / 2; i += NT) v2[i] = lds2[i];
  for (int i = tid; i < sm.nn; i += NT)
    reinterpret_cast<double2*>(rhs_g)[i] = reinterpret_cast<const double2*>(rhs)[i];
  if (bad) d.status[(int64_t)s * (d.n_area + 1) + k] = 1;
}

// ---------------------------------------------------------------------------
// Stage 3a: boundary assembly (Eq. 11).  Each slot of the boundary system's
// packed storage pulls the S_b^k blocks that land on it (E_k as index
// lists); each boundary bus pulls its bhat_b^k entries.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gamma_gather(Dev d, int s0, int nslot) {
  const int s = s0 + blockIdx.y;
  if (!d.active[s]) return;
  const SysMeta g = d.sys[d.n_area];
  const double* base = d.vals + (int64_t)s * d.vstride;
  double* G = d.vals + (int64_t)s * d.vstride + g.val_off;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nslot) {
    const int4 sl = d.g_slot[i];
    double c00 = 0, c10 = 0, c01 = 0, c11 = 0;
    for (int c = sl.z; c < sl.w; ++c) {
      const int4 cc = d.g_con[c];
      const double* S = base + cc.x;
      const double m00 = S[0], m10 = S[1], m01 = S[cc.y], m11 = S[cc.y + 1];
      c00 += m00;
      c11 += m11;
      if (cc.z) { c10 += m01; c01 += m10; }
      else { c10 += m10; c01 += m01; }
    }
    const bool diag = sl.y < 0;
    const int stride = diag ? -sl.y : sl.y;
    if (diag) c01 = c10;
    if (sl.x == g.pin_off) { c00 = 1.0; c10 = 0.0; c01 = 0.0; }
    double* o = G + sl.x;
    o[0] = c00;
    o[1] = c10;
    o[stride] = c01;
    o[stride + 1] = c11;
  }
  if (i < g.nn) {
    const double* rb = d.rhs + (int64_t)s * d.rstride;
    const int2 rs = d.g_rslot[i];
    double b0 = 0, b1 = 0;
    for (int c = rs.x; c < rs.y; ++c) {
      b0 += rb[d.g_rcon[c]];
      b1 += rb[d.g_rcon[c] + 1];
    }
    double* rg = d.rhs + (int64_t)s * d.rstride + g.rhs_off;
    rg[2 * i] = b0;
    rg[2 * i + 1] = b1;
  }
}

// ---------------------------------------------------------------------------
// Stage 3b: dense Cholesky and solve of the boundary system's trailing block
// (the whole S_Gamma in dense mode).  One workgroup per snapshot, blocked
// right-looking with 16-wide panels: the 16x16 diagonal block is factored by
// one wave (wave_chol16_inv4, which also forms its inverse), the panel below
// is multiplied by that inverse on MFMA, and the symmetric trailing update
// A_ij -= L_ik L_jk^T runs on v_mfma_f64_16x16x4f64, one 16x16 tile per wave.
// With one step of lookahead: the next panel's column is updated first, then
// wave 0 factors the next diagonal block while the other waves finish the
// trailing update (every tile still takes the updates in step order).
// The forward solve rides along; the back solve runs block by block from the
// bottom.  The block is column-major with leading dimension n (a multiple of
// 16); rows and columns past the live size are set to the identity first.
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int DENSE_NT = 1024;
constexpr int PANEL_PITCH = 17;  // doubles per staged panel row (odd: no LDS bank conflicts)

// Back substitution L^T x = y of the dense block after its factorisation
// (column-major, leading dimension n, a multiple of 16; y in LDS yv, replaced
// by x), 16-row blocks from the bottom.  With n <= NT - 64 it runs
// right-looking: thread 64 + r owns row r and its running sum acc_r = sum over
// the solved blocks J of L[J][r] . x_J; the 16 entries L[c0 .. c0+15][r] it
// needs for block c0 are contiguous in column r and are loaded one block
// ahead.  Per block, the owners of its rows hand y_r - acc_r to wave 0
// through LDS, wave 0 solves the block's 16 x 16 triangle (loaded one block
// ahead as well), and every owner of a row above adds its 16 products.  Only
// LDS traffic and barriers remain on the chain.  Larger blocks take the
// left-looking form (partial dot products of the columns below each block).
template <int NT>
__device__ __attribute__((always_inline)) inline void dense_back_subst(const double* A, int n, double* yv,
                                                                        double* part, double* xb) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = n / 16;
  if (n > NT - 64) {
    for (int k = nb - 1; k >= 0; --k) {
      const int c0 = 16 * k;
      if (tid < 256) {
        const int c = tid >> 4, pp = tid & 15;  // 16 lanes read 16 consecutive rows of column c
        double acc = 0.0;
        for (int r = c0 + 16 + pp; r < n; r += 16) acc += A[(int64_t)(c0 + c) * n + r] * yv[r];
        part[pp * 16 + c] = acc;
      }
      __syncthreads();
      if (wv == 0) {
        // lane r (mod 16) holds t_r and column r of L_kk
        const int r = lane & 15;
        double col[16];
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) col[mm] = (mm >= r) ? A[(int64_t)(c0 + r) * n + c0 + mm] : 0.0;
        double t = yv[c0 + r];
        for (int pp = 0; pp < 16; ++pp) t -= part[pp * 16 + r];
#pragma unroll
        for (int c = 15; c >= 0; --c) {
          if (r == c) t /= col[c];
          const double xc = bcast_lane(t, c);
          if (r < c) t -= col[c] * xc;
        }
        if (lane < 16) yv[c0 + r] = t;
      }
      __syncthreads();
    }
    return;
  }
  if (wv == 0) {
    // lane q (mod 16) holds t_q, column q of the block's L and 1 / L_qq
    const int q = lane & 15;
    double col[16];
    int c0 = n - 16;
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) col[mm] = (mm >= q) ? A[(int64_t)(c0 + q) * n + c0 + mm] : 0.0;
    double rd = 1.0 / col[q];
    for (int k = nb - 1; k >= 0; --k, c0 -= 16) {
      lds_barrier();  // the owners' t of this block are in xb
      double t = xb[q];
      double cur[16];
#pragma unroll
      for (int mm = 0; mm < 16; ++mm) cur[mm] = col[mm];
      if (k > 0) {
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) col[mm] = (mm >= q) ? A[(int64_t)(c0 - 16 + q) * n + c0 - 16 + mm] : 0.0;
      }
#pragma unroll
      for (int c = 15; c >= 0; --c) {
        if (q == c) t *= rd;
        const double xc = bcast_lane(t, c);
        if (q < c) t -= cur[c] * xc;
      }
      if (lane < 16) {
        yv[c0 + q] = t;
        xb[16 + q] = t;
      }
      lds_barrier();  // x of this block is in xb
      // the next block's reciprocal while the owners add their products
      if (k > 0) rd = 1.0 / col[q];
    }
  } else {
    const int r = tid - 64;
    const bool own = r < n;
    const double* Ar = A + (int64_t)(own ? r : 0) * n;  // column r
    double pf[16];
    double acc = 0.0;
    int c0 = n - 16;
#pragma unroll
    for (int i = 0; i < 16; ++i) pf[i] = (own && r < c0) ? Ar[c0 + i] : 0.0;
    for (int k = nb - 1; k >= 0; --k, c0 -= 16) {
      if (own && r >= c0 && r < c0 + 16) xb[r - c0] = yv[r] - acc;
      lds_barrier();
      lds_barrier();
      if (own && r < c0) {
#pragma unroll
        for (int i = 0; i < 16; ++i) acc += pf[i] * xb[16 + i];
        if (r < c0 - 16) {
#pragma unroll
          for (int i = 0; i < 16; ++i) pf[i] = Ar[c0 - 16 + i];
        }
      }
    }
  }
  __syncthreads();
}

template <bool LDS_PANEL>
__global__ void __launch_bounds__(DENSE_NT) k_dense_chol(Dev d, int s0) {
  const int s = s0 + blockIdx.x;
  if (!d.active[s]) return;
  const SysMeta g = d.sys[d.n_area];
  const int n = g.ld;
  if (n == 0) return;
  const int nlive = 2 * g.nt;
  double* A = d.vals + (int64_t)s * d.vstride + g.val_off + g.tail_off;
  double* b = d.rhs + (int64_t)s * d.rstride + g.rhs_off + 2 * g.ne;
  extern __shared__ double bl[];  // [n] rhs, then solution; then the staged panel
  double* Lp = bl + n;            // [n - 16][PANEL_PITCH]: rows below the diagonal block
  __shared__ double Dk[16 * 17];    // diagonal block, column-major, pitch 17
  __shared__ double Linv[16 * 17];  // its inverse factor, row-major
  __shared__ double cxb[128];
  __shared__ double part[16 * 16];
  __shared__ int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (tid == 0) bad = 0;
  for (int i = tid; i < n; i += nt) bl[i] = (i < nlive) ? b[i] : 0.0;
  // identity padding (lower triangle of the padded rows / columns)
  for (int c = tid; c < n; c += nt)
    for (int r = (c > nlive ? c : nlive); r < n; ++r) A[(int64_t)c * n + r] = (r == c) ? 1.0 : 0.0;
  __syncthreads();
  const int nb = n / 16;
  // the diagonal block of step k to LDS, then wave 0 factors it, solves y
  // and inverts L_kk (the caller synchronises before and after)
  auto load_diag = [&](int k, int first, int stride) {
    const int c0 = 16 * k;
    for (int i = first; i < 256; i += stride) {
      const int r = i & 15, m = i >> 4;
      Dk[m * 17 + r] = (r >= m) ? A[(int64_t)(c0 + m) * n + c0 + r] : 0.0;
    }
  };
  // A_IJ -= L_Ik L_Jk^T for the 16x16 tile at rows ri, columns rj (global
  // offsets), computed transposed (rows J x rows I): lane li holds row ri + li,
  // so the accumulator's global accesses run down a column.
  // v_mfma_f64_16x16x4f64 operands: lane l holds A[l%16][l/16] and
  // B[l/16][l%16]; accumulator element q of lane l is D[4q + l/16][l%16].
  auto tile_load = [&](int ri, int rj, d4& acc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = A[(int64_t)(rj + 4 * q + lk) * n + ri + li];
  };
  auto tile_update = [&](int c0, int ri, int rj, d4& acc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double a, bb;
      if (LDS_PANEL) {
        a = -Lp[(rj - c0 - 16 + li) * PANEL_PITCH + 4 * q + lk];
        bb = Lp[(ri - c0 - 16 + li) * PANEL_PITCH + 4 * q + lk];
      } else {
        a = -A[(int64_t)(c0 + 4 * q + lk) * n + rj + li];
        bb = A[(int64_t)(c0 + 4 * q + lk) * n + ri + li];
      }
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) A[(int64_t)(rj + 4 * q + lk) * n + ri + li] = acc[q];
  };
  // step 0's diagonal block
  load_diag(0, tid, nt);
  __syncthreads();
  if (wv == 0) {
    const bool ok = wave_chol16_inv4(Dk, 17, 0, bl, Linv, cxb);
    if (!ok && lane == 0) bad = 1;
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const int c0 = 16 * k;
    // (1) L_kk back to the block; rows below: X^T = L_kk^-1 A^T on MFMA, one
    // 16-row tile per wave; lane li holds row ri + li, so the accesses run
    // down columns
    for (int i = tid; i < 256; i += nt) {
      const int r = i & 15, m = i >> 4;
      if (r >= m) A[(int64_t)(c0 + m) * n + c0 + r] = Dk[m * 17 + r];
    }
    for (int t = wv; t < nb - k - 1; t += nw) {
      const int ri = c0 + 16 + 16 * t;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double a = Linv[li * 17 + 4 * e + lk];
        const double bb = A[(int64_t)(c0 + 4 * e + lk) * n + ri + li];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        A[(int64_t)(c0 + 4 * e + lk) * n + ri + li] = acc[e];
        if (LDS_PANEL) Lp[(ri + li - c0 - 16) * PANEL_PITCH + 4 * e + lk] = acc[e];
      }
    }
    __syncthreads();
    if (k + 1 == nb) break;
    // (2) rhs of the rows below, and the next panel's column of tiles
    // (I, k + 1), I > k, which the next diagonal factorisation needs first
    for (int row = c0 + 16 + tid; row < n; row += nt) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        acc += (LDS_PANEL ? Lp[(row - c0 - 16) * PANEL_PITCH + c] : A[(int64_t)(c0 + c) * n + row]) * bl[c0 + c];
      bl[row] -= acc;
    }
    for (int t = wv; t < nb - k - 1; t += nw) {
      const int ri = c0 + 16 + 16 * t, rj = c0 + 16;
      d4 acc;
      tile_load(ri, rj, acc);
      tile_update(c0, ri, rj, acc);
    }
    __syncthreads();
    // (3) lookahead: wave 0 factors the next diagonal block while the other
    // waves finish this step's trailing update, tiles (I, J) with
    // k + 1 < J <= I; each wave loads TB tiles together so the global round
    // trips overlap. Every tile still takes the steps' updates in step order.
    if (wv == 0) {
      // the next diagonal block is this phase's critical path: its wave gets
      // the issue slots of its SIMD first
      __builtin_amdgcn_s_setprio(3);
      load_diag(k + 1, lane, 64);
      wave_lds_sync();
      const bool ok = wave_chol16_inv4(Dk, 17, 0, bl + c0 + 16, Linv, cxb);
      if (!ok && lane == 0) bad = 1;
      __builtin_amdgcn_s_setprio(0);
    } else {
      const int m = nb - k - 2;
      const int ntile = m * (m + 1) / 2;
      constexpr int TB = 4;
      const int nwt = nw - 1;
      for (int t0 = wv - 1; t0 < ntile; t0 += nwt * TB) {
        int ri[TB], rj[TB];
        d4 acc[TB];
#pragma unroll
        for (int bq = 0; bq < TB; ++bq) {
          const int t = t0 + bq * nwt;
          ri[bq] = -1;
          if (t < ntile) {
            int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
            while (I * (I + 1) / 2 > t) --I;
            while ((I + 1) * (I + 2) / 2 <= t) ++I;
            const int J = t - I * (I + 1) / 2;
            ri[bq] = 16 * (k + 2 + I);
            rj[bq] = 16 * (k + 2 + J);
            tile_load(ri[bq], rj[bq], acc[bq]);
          }
        }
#pragma unroll
        for (int bq = 0; bq < TB; ++bq)
          if (ri[bq] >= 0) tile_update(c0, ri[bq], rj[bq], acc[bq]);
      }
    }
    __syncthreads();
  }
  __syncthreads();
  dense_back_subst<DENSE_NT>(A, n, bl, part, cxb);
  for (int i = tid; i < nlive; i += nt) b[i] = bl[i];
  if (tid == 0 && bad) d.status[(int64_t)s * (d.n_area + 1) + d.n_area] = 1;
}

// ---------------------------------------------------------------------------
// Stage 3b, wide panels: the same factorisation and solve with nb-column
// panels (nb a multiple of 16, up to 64) staged whole in LDS.  A panel is
// factored there in 16-column steps (wave-level 16x16 Cholesky with its
// inverse, rows below on MFMA, the panel's later columns updated on MFMA),
// written back, and the trailing matrix then takes one rank-nb update on
// MFMA: nb/16 times fewer read-modify-write rounds over the trailing matrix
// in HBM than 16-column steps need.  The rhs stays in LDS throughout.
// ---------------------------------------------------------------------------
constexpr int DW_NT = 1024;

__global__ void __launch_bounds__(DW_NT) k_dense_wide(Dev d, int s0, int nb) {
  const int s = s0 + blockIdx.x;
  if (!d.active[s]) return;
  const SysMeta g = d.sys[d.n_area];
  const int n = g.ld;
  if (n == 0) return;
  const int nlive = 2 * g.nt;
  double* A = d.vals + (int64_t)s * d.vstride + g.val_off + g.tail_off;
  double* b = d.rhs + (int64_t)s * d.rstride + g.rhs_off + 2 * g.ne;
  extern __shared__ double dw[];
  double* yv = dw;      // [n] rhs, then the solution
  double* P = dw + n;   // [nb columns][M rows] of the current panel, M = n - c0, pitch M + 1
  __shared__ double Linv[16 * 17];
  __shared__ double cxb[128];
  __shared__ double part[16 * 16];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = DW_NT / 64, TB = 4, UL = 8;
  const int li = lane & 15, lk = lane >> 4;
  if (tid == 0) bad = 0;
  for (int i = tid; i < n; i += DW_NT) yv[i] = (i < nlive) ? b[i] : 0.0;
  // identity padding (lower triangle of the padded rows / columns)
  for (int c = tid; c < n; c += DW_NT)
    for (int r = (c > nlive ? c : nlive); r < n; ++r) A[(int64_t)c * n + r] = (r == c) ? 1.0 : 0.0;
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += nb) {
    const int w = min(nb, n - c0), M = n - c0, ldp = M + 1;  // odd pitch: columns in distinct banks
    const double invM = 1.0 / M;
    // (1) stage the panel's lower part, UL loads in flight per thread
    for (int i0 = tid; i0 < w * M; i0 += UL * DW_NT) {
      double v[UL];
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int i = i0 + u * DW_NT;
        const int col = (int)((i + 0.5) * invM), row = i - col * M;
        v[u] = (i < w * M && row >= col) ? A[(int64_t)(c0 + col) * n + c0 + row] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int i = i0 + u * DW_NT;
        const int col = (int)((i + 0.5) * invM), row = i - col * M;
        if (i < w * M) P[col * ldp + row] = v[u];
      }
    }
    __syncthreads();
    // (2) factor the panel in 16-column steps
    for (int cb = 0; cb < w; cb += 16) {
      if (wv == 0) {
        const bool ok = wave_chol16_inv4(P, ldp, cb, yv + c0, Linv, cxb);
        if (!ok && lane == 0) bad = 1;
      }
      __syncthreads();
      // rows below the block: X = A L^-T, one 16-row tile per wave, on MFMA
      const int rt0 = cb / 16 + 1, nrt = M / 16 - rt0;
      for (int t = wv; t < nrt; t += NW) {
        const int ri = 16 * (rt0 + t);
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double a = P[(cb + 4 * e + lk) * ldp + ri + li];
          const double bb = Linv[li * 17 + 4 * e + lk];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) P[(cb + li) * ldp + ri + 4 * e + lk] = acc[e];
      }
      __syncthreads();
      // rhs of the rows below, and the panel's remaining columns
      for (int row = cb + 16 + tid; row < M; row += DW_NT) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 16; ++c) acc += P[(cb + c) * ldp + row] * yv[c0 + cb + c];
        yv[c0 + row] -= acc;
      }
      const int jt0 = cb / 16 + 1, njt = w / 16 - jt0, nrt2 = M / 16;
      int ntile = 0;
      for (int j = 0; j < njt; ++j) ntile += nrt2 - (jt0 + j);
      for (int t = wv; t < ntile; t += NW) {
        int j = 0, tt = t;
        while (tt >= nrt2 - (jt0 + j)) {
          tt -= nrt2 - (jt0 + j);
          ++j;
        }
        const int rj = 16 * (jt0 + j), ri = rj + 16 * tt;
        d4 acc;
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = P[(rj + li) * ldp + ri + 4 * e + lk];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double a = -P[(cb + 4 * e + lk) * ldp + ri + li];
          const double bb = P[(cb + 4 * e + lk) * ldp + rj + li];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) P[(rj + li) * ldp + ri + 4 * e + lk] = acc[e];
      }
      __syncthreads();
    }
    // (3) the factor back to HBM (lower part)
    for (int i = tid; i < w * M; i += DW_NT) {
      const int col = (int)((i + 0.5) * invM), row = i - col * M;
      if (row >= col) A[(int64_t)(c0 + col) * n + c0 + row] = P[col * ldp + row];
    }
    // (4) trailing update A_IJ -= L_I L_J^T over the rows below the panel:
    // tiles (I >= J); a wave loads TB tiles, updates them, stores them
    const int mt = (M - w) / 16, ntile = mt * (mt + 1) / 2;
    for (int t0 = wv; t0 < ntile; t0 += NW * TB) {
      int ri[TB], rj[TB];
      d4 acc[TB];
#pragma unroll
      for (int bq = 0; bq < TB; ++bq) {
        const int t = t0 + bq * NW;
        ri[bq] = -1;
        if (t < ntile) {
          int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
          while (I * (I + 1) / 2 > t) --I;
          while ((I + 1) * (I + 2) / 2 <= t) ++I;
          const int J = t - I * (I + 1) / 2;
          ri[bq] = w + 16 * I;
          rj[bq] = w + 16 * J;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            acc[bq][q] = A[(int64_t)(c0 + rj[bq] + 4 * q + lk) * n + c0 + ri[bq] + li];
        }
      }
#pragma unroll
      for (int bq = 0; bq < TB; ++bq) {
        if (ri[bq] < 0) continue;
        // computed transposed (rows J x rows I): lane li holds row ri + li,
        // so the accumulator's global accesses run down a column
        for (int k4 = 0; k4 < w; k4 += 4) {
          const double a = -P[(k4 + lk) * ldp + rj[bq] + li];
          const double bb = P[(k4 + lk) * ldp + ri[bq] + li];
          acc[bq] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc[bq], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) A[(int64_t)(c0 + rj[bq] + 4 * q + lk) * n + c0 + ri[bq] + li] = acc[bq][q];
      }
    }
    __syncthreads();
  }
  __syncthreads();
  dense_back_subst<DW_NT>(A, n, yv, part, cxb);
  for (int i = tid; i < nlive; i += DW_NT) b[i] = yv[i];
  if (tid == 0 && bad) d.status[(int64_t)s * (d.n_area + 1) + d.n_area] = 1;
}

// ---------------------------------------------------------------------------
// Stage 3b (sparse part, supernodal): elimination of the boundary system's
// leading buses one supernode at a time (one workgroup per snapshot).  A
// supernode is a run of buses whose factor columns share the row list R below
// their diagonal block, so the run is one dense panel: its 2w own variables
// (padded to a multiple of 16 with an identity) and the 2r variables of R.
// Per supernode: (1) the panel's columns, which are contiguous in the packed
// storage, its rhs and its target offsets are staged in LDS; (2) blocked
// Cholesky of the panel in 16-column steps (wave 0 factors the 16x16
// diagonal block in registers, every thread solves one row of the blocks
// below, the remaining panel columns are updated on FP64 MFMA) together with
// the forward solve of the rhs; (3) the Schur update L_R L_R^T of the R x R
// blocks, on FP64 MFMA, is subtracted from the packed storage, whose blocks
// (R[a], R[c]) the plan lists; (4) the factor is written back.  Diagonal 2x2
// blocks are written as L_jj L_jj^T, the fully updated pivot block, which is
// the form the level-scheduled back substitution reads (Eq. 8-11).
// ---------------------------------------------------------------------------
constexpr int SN_NT = 512;

// Panel coordinates of element i of a supernode's packed columns: column bus
// b of w, block kk of that column (0: the diagonal block, then the own buses
// below it, then R), element e of the column-major 2x2 block.
// Column b starts at f(b) = 4 b (w + r) - 2 b (b - 1) = b (B - 2 b) with
// B = 4 (w + r) + 2, increasing in b; b is found by binary search (w <= 32).
__device__ inline void sn_coords(int i, int w, int r, int Wp, int& rowv, int& colv, int& kk, int& e,
                                 int& bb) {
  const int B = 4 * (w + r) + 2;
  int lo = 0, hi = w - 1;  // largest b with f(b) <= i
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    const int mid = (lo + hi + 1) >> 1;
    const bool le = mid * (B - 2 * mid) <= i;
    lo = le ? mid : lo;
    hi = le ? hi : mid - 1;
  }
  bb = lo;
  const int st = bb * (B - 2 * bb);
  kk = (i - st) >> 2;
  e = (i - st) & 3;
  const int u = e & 1, v = e >> 1;
  rowv = (kk <= w - 1 - bb) ? 2 * (bb + kk) + u : Wp + 2 * (kk - (w - bb)) + u;
  colv = 2 * bb + v;
}

// One workgroup per (snapshot, group of elimination subtrees): subtrees that
// hang off different points of the tail share no factor entries below it, so
// their groups run side by side.  What they do share, the tail block and the
// tail rhs, is left alone here: each supernode stores its update of them,
// U_q = L_T L_T^T over its tail rows T and c_q = -L_T y_q, and k_gamma_tail
// applies them afterwards.
__global__ void __launch_bounds__(SN_NT) k_gamma_snode(Dev d, int s0) {
  const int gi = blockIdx.x % d.n_sn_grp;
  const int s = s0 + blockIdx.x / d.n_sn_grp;
  if (!d.active[s]) return;
  const SysMeta g = d.sys[d.n_area];
  double* vals = d.vals + (int64_t)s * d.vstride + g.val_off;
  double* rhs = d.rhs + (int64_t)s * d.rstride + g.rhs_off;
  double* tl = d.sn_tl + (int64_t)s * d.tl_stride;
  extern __shared__ double sl[];
  __shared__ double Linv[16 * 17];
  __shared__ double cxb[128];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = SN_NT / 64, UL = 8, TB = 4;
  const int li = lane & 15, lk = lane >> 4;
  if (tid == 0) bad = 0;
  const int qb = d.sn_grp_ptr[gi], qe = d.sn_grp_ptr[gi + 1];
  // the plan records of the group's next supernode are fetched while the
  // current one is factored
  int4 snx = make_int4(0, 0, 0, 0), sn2x = make_int4(0, 0, 0, 0);
  if (qb < qe) {
    const int q0 = d.sn_grp[qb];
    snx = d.sn[q0];
    sn2x = d.sn2[q0];
  }
  for (int qi = qb; qi < qe; ++qi) {
    const int q = d.sn_grp[qi];
    const int qn = (qi + 1 < qe) ? d.sn_grp[qi + 1] : 0;
    const int4 sn = snx;
    const int4 sn2 = sn2x;
    const int c0 = sn.x, w = sn.y, r = sn.z, rb = sn.w;
    const int nrs = r - sn2.w;  // R buses outside the tail
    const int W = 2 * w, Wp = (W + 15) & ~15, M = Wp + ((2 * r + 15) & ~15);
    const int ldp = M + 1;  // odd pitch: the panel's columns start in distinct LDS banks
    const int T = sn2.y, ntg = r * (r + 1) / 2;
    double* P = sl;              // [Wp columns][M rows], pitch ldp
    double* yv = sl + ldp * Wp;  // [M]
    int* tg = reinterpret_cast<int*>(yv + M);
    int* rows = tg + ntg;        // [r] the R bus ids
    // (1) staging.  Every load of the stage is issued first (the panel's
    // first UL values per thread, the own rhs, the R bus ids, the target
    // table), the LDS is cleared meanwhile (a barrier on LDS alone keeps
    // them in flight), and only the rhs of the R rows, which needs the bus
    // ids, waits for a first round trip.
    double v[UL];
#pragma unroll
    for (int u = 0; u < UL; ++u) {
      const int i = tid + u * SN_NT;
      v[u] = (i < T) ? vals[sn2.x + i] : 0.0;
    }
    const double yown = tid < W ? rhs[2 * c0 + tid] : 0.0;
    const int rid = tid < r ? d.sn_rows[rb + tid] : 0;
    int tgv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) tgv[u] = (tid + u * SN_NT < ntg) ? d.sn_tgt[sn2.z + tid + u * SN_NT] : 0;
    for (int i = tid; i < ldp * Wp; i += SN_NT) P[i] = 0.0;
    for (int i = tid; i < M; i += SN_NT) yv[i] = 0.0;
    lds_barrier();
    if (tid < r) rows[tid] = rid;
    for (int i = tid + SN_NT; i < r; i += SN_NT) rows[i] = d.sn_rows[rb + i];
    if (tid < Wp - W) P[(W + tid) * ldp + W + tid] = 1.0;
    if (tid < W) yv[tid] = yown;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (tid + u * SN_NT < ntg) tg[tid + u * SN_NT] = tgv[u];
    for (int i = tid + 4 * SN_NT; i < ntg; i += SN_NT) tg[i] = d.sn_tgt[sn2.z + i];
    for (int i0 = tid; i0 < T; i0 += UL * SN_NT) {
      if (i0 != tid) {
#pragma unroll
        for (int u = 0; u < UL; ++u) {
          const int i = i0 + u * SN_NT;
          v[u] = (i < T) ? vals[sn2.x + i] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int i = i0 + u * SN_NT;
        if (i >= T) break;
        int rowv, colv, kk, e, bb;
        sn_coords(i, w, r, Wp, rowv, colv, kk, e, bb);
        if (kk == 0 && e == 2) continue;  // upper entry of the diagonal block
        P[colv * ldp + rowv] = v[u];
      }
    }
    if (qi + 1 < qe) {
      snx = d.sn[qn];
      sn2x = d.sn2[qn];
    }
    lds_barrier();
    for (int i = tid; i < 2 * nrs; i += SN_NT) yv[Wp + i] = rhs[2 * rows[i >> 1] + (i & 1)];
    __syncthreads();
    // (2) blocked Cholesky of the panel and forward solve
    for (int cb = 0; cb < Wp; cb += 16) {
      if (wv == 0) {
        const bool ok = wave_chol16_inv4(P, ldp, cb, yv, Linv, cxb);
        if (!ok && lane == 0) bad = 1;
      }
      __syncthreads();
      // rows below the block: X = A L^-T, one 16-row tile per wave, on MFMA
      const int rt0 = cb / 16 + 1, nrt = M / 16 - rt0;
      for (int t = wv; t < nrt; t += NW) {
        const int ri = 16 * (rt0 + t);
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double a = P[(cb + 4 * e + lk) * ldp + ri + li];
          const double bb = Linv[li * 17 + 4 * e + lk];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) P[(cb + li) * ldp + ri + 4 * e + lk] = acc[e];
      }
      __syncthreads();
      // rhs of the rows below, and the remaining panel columns: tiles
      // (row tile ic >= column tile jc > cb / 16)
      for (int row = cb + 16 + tid; row < M; row += SN_NT) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 16; ++c) acc += P[(cb + c) * ldp + row] * yv[cb + c];
        yv[row] -= acc;
      }
      const int jt0 = cb / 16 + 1, njt = Wp / 16 - jt0, nrt2 = M / 16;
      int ntile = 0;
      for (int j = 0; j < njt; ++j) ntile += nrt2 - (jt0 + j);
      for (int t = wv; t < ntile; t += NW) {
        int j = 0, tt = t;
        while (tt >= nrt2 - (jt0 + j)) {
          tt -= nrt2 - (jt0 + j);
          ++j;
        }
        const int rj = 16 * (jt0 + j), ri = rj + 16 * tt;
        d4 acc;
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = P[(rj + li) * ldp + ri + 4 * e + lk];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double a = -P[(cb + 4 * e + lk) * ldp + ri + li];
          const double bb = P[(cb + 4 * e + lk) * ldp + rj + li];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) P[(rj + li) * ldp + ri + 4 * e + lk] = acc[e];
      }
      __syncthreads();
    }
    // (3) factor and forward-solved rhs back to HBM (issued before the Schur
    // update, so that the stores drain while it computes)
    for (int i = tid; i < T; i += SN_NT) {
      int rowv, colv, kk, e, bb;
      sn_coords(i, w, r, Wp, rowv, colv, kk, e, bb);
      double val;
      if (kk == 0) {
        const double l00 = P[(2 * bb) * ldp + 2 * bb], l10 = P[(2 * bb) * ldp + 2 * bb + 1];
        const double l11 = P[(2 * bb + 1) * ldp + 2 * bb + 1];
        val = (e == 0) ? l00 * l00 : (e == 3) ? l10 * l10 + l11 * l11 : l10 * l00;
      } else {
        val = P[colv * ldp + rowv];
      }
      vals[sn2.x + i] = val;
    }
    for (int i = tid; i < W; i += SN_NT) rhs[2 * c0 + i] = yv[i];
    for (int i = tid; i < 2 * nrs; i += SN_NT) rhs[2 * rows[i >> 1] + (i & 1)] = yv[Wp + i];
    const int mt = 2 * sn2.w;  // tail rows: their rhs started at 0, so they now hold c_q
    const int4 s3 = d.sn3[q];
    for (int i = tid; i < mt; i += SN_NT) tl[s3.y + i] = yv[Wp + 2 * nrs + i];
    // (4) Schur update of the R x R blocks: tiles (I >= J) of the R rows.
    // Targets outside the tail block are read, updated and written back (a
    // wave computes TB tiles, then loads all their targets, then stores, so
    // the round trips overlap); the tail block's part is stored as U_q.
    const int nr = (M - Wp) / 16, nt3 = nr * (nr + 1) / 2;
    for (int t0 = wv; t0 < nt3; t0 += NW * TB) {
      d4 acc[TB];
      int idx[TB][4];
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int t = t0 + b * NW;
#pragma unroll
        for (int e = 0; e < 4; ++e) idx[b][e] = -1;
        if (t >= nt3) continue;
        int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while (I * (I + 1) / 2 > t) --I;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        const int J = t - I * (I + 1) / 2;
        // the tile is computed transposed (D = rows J x rows I): lane li then
        // holds row 16 I + li, so lanes run down a column of the target
        const int ri = Wp + 16 * I, rj = Wp + 16 * J;
        acc[b] = d4{0.0, 0.0, 0.0, 0.0};
        for (int k4 = 0; k4 < Wp; k4 += 4) {
          const double a = P[(k4 + lk) * ldp + rj + li];
          const double bb = P[(k4 + lk) * ldp + ri + li];
          acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc[b], 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int xv = 16 * I + li, yc = 16 * J + 4 * e + lk;
          const int ab = xv >> 1, cb2 = yc >> 1;
          if (xv < 2 * r && yc < 2 * r && ab >= cb2) {
            if (cb2 < nrs)
              idx[b][e] = tg[ab * (ab + 1) / 2 + cb2] + (xv & 1) + 2 * (yc & 1);
            else
              tl[s3.x + (yc - 2 * nrs) * mt + (xv - 2 * nrs)] = acc[b][e];
          }
        }
      }
      double old[TB][4];
#pragma unroll
      for (int b = 0; b < TB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) old[b][e] = (idx[b][e] >= 0) ? vals[idx[b][e]] : 0.0;
#pragma unroll
      for (int b = 0; b < TB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (idx[b][e] >= 0) vals[idx[b][e]] = old[b][e] - acc[b][e];
    }
    __syncthreads();
  }
  if (tid == 0 && bad) d.status[(int64_t)s * (d.n_area + 1) + d.n_area] = 1;
}

// ---------------------------------------------------------------------------
// Stage 3c, supernodal back substitution of the boundary system's leading
// buses (Eq. 8-11 through the cached factor), after the dense block has been
// solved: one workgroup per (snapshot, subtree group), the group's supernodes
// from the top down.  Per supernode the panel is staged in LDS (diagonal 2x2
// blocks, stored as L_jj L_jj^T, are factored again), then
// t = y_own - L_R^T x_R with x_R the solution of its row buses (tail or
// ancestors in the same subtree, both final), and L_own^T x_own = t is solved
// by one wave, one variable per lane.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(SN_NT) k_gamma_snode_back(Dev d, int s0) {
  const int gi = blockIdx.x % d.n_sn_grp;
  const int s = s0 + blockIdx.x / d.n_sn_grp;
  if (!d.active[s]) return;
  const SysMeta g = d.sys[d.n_area];
  const double* vals = d.vals + (int64_t)s * d.vstride + g.val_off;
  double* rhs = d.rhs + (int64_t)s * d.rstride + g.rhs_off;
  extern __shared__ double sl[];
  __shared__ double part[8 * 64];
  __shared__ double tv[64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int UL = 8;
  const int qb = d.sn_grp_ptr[gi];
  for (int qi = d.sn_grp_ptr[gi + 1] - 1; qi >= qb; --qi) {
    const int q = d.sn_grp[qi];
    const int4 sn = d.sn[q];
    const int4 sn2 = d.sn2[q];
    const int c0 = sn.x, w = sn.y, r = sn.z, rb = sn.w;
    const int W = 2 * w, Wp = (W + 15) & ~15, M = Wp + ((2 * r + 15) & ~15);
    const int ldp = M + 1;
    const int T = sn2.y;
    double* P = sl;              // [Wp columns][M rows], pitch ldp
    double* xr = sl + ldp * Wp;  // [2 r] solution of the row buses
    // (1) staging of the panel's stored factor
    for (int i0 = tid; i0 < T; i0 += UL * SN_NT) {
      double v[UL];
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int i = i0 + u * SN_NT;
        v[u] = (i < T) ? vals[sn2.x + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int i = i0 + u * SN_NT;
        if (i >= T) break;
        int rowv, colv, kk, e, bb;
        sn_coords(i, w, r, Wp, rowv, colv, kk, e, bb);
        if (kk == 0 && e == 2) continue;  // upper entry of the diagonal block
        P[colv * ldp + rowv] = v[u];
      }
    }
    for (int i = tid; i < 2 * r; i += SN_NT) xr[i] = rhs[2 * d.sn_rows[rb + (i >> 1)] + (i & 1)];
    if (tid < W) tv[tid] = rhs[2 * c0 + tid];
    __syncthreads();
    // diagonal blocks back from L_jj L_jj^T to L_jj
    if (tid < w) {
      const int j = 2 * tid;
      double l00, l10, l11;
      if (!chol2(P[j * ldp + j], P[j * ldp + j + 1], P[(j + 1) * ldp + j + 1], l00, l10, l11)) {
        l00 = l11 = 1.0;
        l10 = 0.0;
      }
      P[j * ldp + j] = l00;
      P[j * ldp + j + 1] = l10;
      P[(j + 1) * ldp + j + 1] = l11;
    }
    // (2) t = y_own - L_R^T x_R: column c by 8 threads, fixed-order sum
    {
      const int c = tid & 63, pp = tid >> 6;
      double acc = 0.0;
      if (c < W)
        for (int j = pp; j < 2 * r; j += 8) acc += P[c * ldp + Wp + j] * xr[j];
      part[pp * 64 + c] = acc;
    }
    __syncthreads();
    // (3) L_own^T x = t by wave 0, lane c holding variable c (c < W), from
    // the last variable up
    if (wv == 0) {
      double t = 0.0, rinv = 1.0;
      if (lane < W) {
        t = tv[lane];
        for (int pp = 0; pp < 8; ++pp) t -= part[pp * 64 + lane];
        rinv = 1.0 / P[lane * ldp + lane];
      }
      for (int c = W - 1; c >= 0; --c) {
        if (lane == c) t *= rinv;
        const double xc = bcast_lane(t, c);
        if (lane < c) t -= P[lane * ldp + c] * xc;
      }
      if (lane < W) rhs[2 * c0 + lane] = t;
    }
    __syncthreads();
  }
}

hipError_t launch_gamma_snode_back(const Dev& d, int s0, int ns, size_t lds, hipStream_t st) {
  if (ns <= 0 || d.n_sn <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gamma_snode_back, dim3(ns * d.n_sn_grp), dim3(SN_NT), lds, st, d, s0);
  return hipGetLastError();
}

hipError_t allow_gamma_snode_back_lds(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gamma_snode_back),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ---------------------------------------------------------------------------
// Stage 3b (sparse part, tail updates): every tail entry of the boundary
// system takes the updates the supernodes left for it, A -= U_q and b += c_q,
// in supernode order (the order of a one-workgroup elimination), from a
// fixed contribution list.  One thread per entry.
// ---------------------------------------------------------------------------
constexpr int TAIL_NT = 256;

__global__ void __launch_bounds__(TAIL_NT) k_gamma_tail(Dev d, int s0, int nblk) {
  const int e = (blockIdx.x % nblk) * TAIL_NT + threadIdx.x;
  const int s = s0 + blockIdx.x / nblk;
  if (e >= d.n_tail_ent || !d.active[s]) return;
  const SysMeta g = d.sys[d.n_area];
  const int4 te = d.tail_ent[e];
  const double* tl = d.sn_tl + (int64_t)s * d.tl_stride;
  double* tgt = te.y ? d.rhs + (int64_t)s * d.rstride + g.rhs_off + 2 * g.ne + te.x
                     : d.vals + (int64_t)s * d.vstride + g.val_off + g.tail_off + te.x;
  double v = *tgt;
  int c = te.z;
  // four sources in flight at a time
  for (; c + 4 <= te.w; c += 4) {
    const int o0 = d.tail_con[c], o1 = d.tail_con[c + 1], o2 = d.tail_con[c + 2], o3 = d.tail_con[c + 3];
    const double u0 = tl[o0], u1 = tl[o1], u2 = tl[o2], u3 = tl[o3];
    v = te.y ? v + u0 : v - u0;
    v = te.y ? v + u1 : v - u1;
    v = te.y ? v + u2 : v - u2;
    v = te.y ? v + u3 : v - u3;
  }
  for (; c < te.w; ++c) {
    const double u = tl[d.tail_con[c]];
    v = te.y ? v + u : v - u;
  }
  *tgt = v;
}

// ---------------------------------------------------------------------------
// Stage 4a: back substitution.  For an area, first copy dx of its local
// boundary buses from the boundary solution (dx_b^k = E_k dx_Gamma); then,
// level by level from the top, dx_j = L_jj^-T (y_j - sum_i L_ij^T dx_i),
// which is Eq. 8 through the cached factor.  Each column's sum is split over
// a group of lanes (1 to 64, chosen per level by the plan) and combined by a
// fixed shuffle tree.
// ---------------------------------------------------------------------------
template <int NT, bool XL>
__global__ void __launch_bounds__(NT) k_backsolve(Dev d, int sys0, int nsys, int s0, int ns, int fixed_bnd) {
  int si, s;
  area_snap_of_block(blockIdx.x, nsys, ns, si, s);
  s += s0;
  if (!d.active[s]) return;
  const bool is_area = sys0 < d.n_area;
  const int k = is_area ? d.area_order[sys0 + si] : sys0 + si;
  const SysMeta sm = d.sys[k];
  const double* vals = d.vals + (int64_t)s * d.vstride + sm.val_off;
  double* rb = d.rhs + (int64_t)s * d.rstride;
  double* rhs = rb + sm.rhs_off;
  const int tid = threadIdx.x;
  // the system's rhs lives in LDS for the whole substitution (y in, x out),
  // or stays in HBM when the largest system's does not fit
  extern __shared__ double xlds[];
  double* xl = XL ? xlds : rhs;
  if (XL)
    for (int i = tid; i < 2 * sm.ne; i += NT) xl[i] = rhs[i];
  if (is_area) {
    const AreaMeta am = d.area[k];
    for (int t = tid; t < sm.nt; t += NT) {
      // dx_b = E_k dx_Gamma, or 0 for a local step with the boundary fixed
      const int src = d.tail_src[am.tail_src + t];
      xl[2 * (sm.ne + t)] = fixed_bnd ? 0.0 : rb[src];
      xl[2 * (sm.ne + t) + 1] = fixed_bnd ? 0.0 : rb[src + 1];
    }
  } else if (XL) {
    for (int i = 2 * sm.ne + tid; i < 2 * sm.nn; i += NT) xl[i] = rhs[i];
  }
  __syncthreads();
  // Lanes per column vary by level (2^lg of them, from the plan: many short
  // columns near the leaves, a few long ones near the root); lane gl of a
  // group sums rows gl, gl + G, ... of its column, then the group reduces.
  // The factor is only read here, so every load of a level's first pass (a
  // factor block per lane, the pivot block per group) goes out in one burst
  // together with the next level's first contribution records, the item
  // records two levels ahead and the level bounds three ahead; one wait
  // covers them all.  Loads complete in issue order, so records fetched
  // early are only free if nothing waits in between.  With x in LDS the
  // barriers order LDS only.
  const int32_t* bsp = d.bs_ptr + sm.bs_ptr;
  const int32_t* bsg = d.bs_lg + sm.bs_ptr;
  const int nlev = sm.nlev;
  const Rec4 none{0, 0, 0, 0};
  // this level: items [b0, b1), 2^lg lanes per item; the next level: items
  // [n_b0, b0); the one after: [nn_b0, n_b0)
  int b0 = 0, b1 = 0, lg = 0, n_b0 = 0, n_lg = 0, nn_b0 = 0, nn_lg = 0;
  Rec4 irec = none, n_irec = none;
  Rec2 crec{0, 0};
  if (nlev > 0) {
    b1 = __builtin_amdgcn_readfirstlane(bsp[nlev]);
    b0 = __builtin_amdgcn_readfirstlane(bsp[nlev - 1]);
    lg = __builtin_amdgcn_readfirstlane(bsg[nlev - 1]);
    if (b0 + (tid >> lg) < b1) irec = ld_rec(d.bs_items + b0 + (tid >> lg));
    if (irec.z + (tid & ((1 << lg) - 1)) < irec.w) crec = ld_rec(d.bs_con + irec.z + (tid & ((1 << lg) - 1)));
    if (nlev > 1) {
      n_b0 = __builtin_amdgcn_readfirstlane(bsp[nlev - 2]);
      n_lg = __builtin_amdgcn_readfirstlane(bsg[nlev - 2]);
      if (n_b0 + (tid >> n_lg) < b0) n_irec = ld_rec(d.bs_items + n_b0 + (tid >> n_lg));
    }
    if (nlev > 2) {
      nn_b0 = __builtin_amdgcn_readfirstlane(bsp[nlev - 3]);
      nn_lg = __builtin_amdgcn_readfirstlane(bsg[nlev - 3]);
    }
  }
  for (int lev = nlev - 1; lev >= 0; --lev) {
    const int G = 1 << lg, grp = tid >> lg, gl = tid & (G - 1);
    // ---- the burst
    const bool has_item = b0 + grp < b1;
    double p0 = 0, p1 = 0, p2 = 0, p3 = 0, q0 = 0, q1 = 0, q3 = 0;
    if (has_item && irec.z + gl < irec.w) {
      const double* Lb = vals + crec.x;
      p0 = Lb[0]; p1 = Lb[1]; p2 = Lb[2]; p3 = Lb[3];
    }
    if (has_item && gl == 0) {
      const double* D = vals + irec.x;
      q0 = D[0]; q1 = D[1]; q3 = D[3];
    }
    Rec2 n_crec{0, 0};
    if (lev >= 1) {
      const int ngl = tid & ((1 << n_lg) - 1);
      if (n_b0 + (tid >> n_lg) < b0 && n_irec.z + ngl < n_irec.w) n_crec = ld_rec(d.bs_con + n_irec.z + ngl);
    }
    Rec4 nn_irec = none;
    if (lev >= 2 && nn_b0 + (tid >> nn_lg) < n_b0) nn_irec = ld_rec(d.bs_items + nn_b0 + (tid >> nn_lg));
    int nnn_b0 = 0, nnn_lg = 0;
    if (lev >= 3) {
      nnn_b0 = bsp[lev - 3];
      nnn_lg = bsg[lev - 3];
    }
    // ---- the level's columns
    for (int it = b0 + grp; it < b1; it += NT >> lg) {
      const bool first = it == b0 + grp;
      const Rec4 b = first ? irec : ld_rec(d.bs_items + it);
      double t0 = 0.0, t1 = 0.0;
      for (int c = b.z + gl; c < b.w; c += G) {
        const bool pre = first && c == b.z + gl;
        const Rec2 u = pre ? crec : ld_rec(d.bs_con + c);
        double l0, l1, l2, l3;
        if (pre) {
          l0 = p0; l1 = p1; l2 = p2; l3 = p3;
        } else {
          const double* Lb = vals + u.x;
          l0 = Lb[0]; l1 = Lb[1]; l2 = Lb[2]; l3 = Lb[3];
        }
        const double x0 = xl[u.y], x1 = xl[u.y + 1];
        t0 += l0 * x0 + l1 * x1;
        t1 += l2 * x0 + l3 * x1;
      }
      for (int off = G >> 1; off > 0; off >>= 1) {
        t0 += __shfl_xor(t0, off);
        t1 += __shfl_xor(t1, off);
      }
      if (gl == 0) {
        t0 = xl[b.y] - t0;
        t1 = xl[b.y + 1] - t1;
        double a00, a10, a11;
        if (first) {
          a00 = q0; a10 = q1; a11 = q3;
        } else {
          const double* D = vals + b.x;
          a00 = D[0]; a10 = D[1]; a11 = D[3];
        }
        double l00, l10, l11, i00, i11;
        if (!chol2(a00, a10, a11, l00, l10, l11, i00, i11)) {
          l00 = l11 = i00 = i11 = 1.0;
          l10 = 0.0;
        }
        const double x1 = t1 * i11;
        xl[b.y + 1] = x1;
        xl[b.y] = (t0 - l10 * x1) * i00;
      }
    }
    if constexpr (XL) lds_barrier();
    else __syncthreads();
    b1 = b0; b0 = n_b0; lg = n_lg;
    n_b0 = nn_b0; n_lg = nn_lg;
    nn_b0 = __builtin_amdgcn_readfirstlane(nnn_b0);
    nn_lg = __builtin_amdgcn_readfirstlane(nnn_lg);
    irec = n_irec;
    n_irec = nn_irec;
    crec = n_crec;
  }
  if (XL)
    for (int i = tid; i < 2 * sm.nn; i += NT) rhs[i] = xl[i];
}

// ---------------------------------------------------------------------------
// Stage 4a for an area held in LDS: its factor [0, tail_off) is read once,
// coalesced, into LDS next to the rhs; the level-by-level substitution of
// k_backsolve then runs on LDS only (same arithmetic, same order, so the
// same results).
// ---------------------------------------------------------------------------
template <int NT>
__global__ void __launch_bounds__(NT) k_back_lds(Dev d, int a0, int na, int s0, int ns, int fixed_bnd) {
  int ai, s;
  area_snap_of_block(blockIdx.x, na, ns, ai, s);
  s += s0;
  if (!d.active[s]) return;
  const int k = d.area_order[a0 + ai];
  const SysMeta sm = d.sys[k];
  const AreaMeta am = d.area[k];
  const double* vals = d.vals + (int64_t)s * d.vstride + sm.val_off;
  double* rb = d.rhs + (int64_t)s * d.rstride;
  double* rhs = rb + sm.rhs_off;
  extern __shared__ double2 lds2[];
  double* L = reinterpret_cast<double*>(lds2);
  const int nl = sm.tail_off;  // a multiple of 16
  double* xl = L + nl;
  const int tid = threadIdx.x;
  const double2* v2 = reinterpret_cast<const double2*>(vals);
  for (int i = tid; i < nl / 2; i += NT) lds2[i] = v2[i];
  for (int i = tid; i < 2 * sm.ne; i += NT) xl[i] = rhs[i];
  for (int t = tid; t < sm.nt; t += NT) {
    // dx_b = E_k dx_Gamma, or 0 for a local step with the boundary fixed
    const int src = d.tail_src[am.tail_src + t];
    xl[2 * (sm.ne + t)] = fixed_bnd ? 0.0 : rb[src];
    xl[2 * (sm.ne + t) + 1] = fixed_bnd ? 0.0 : rb[src + 1];
  }
  __syncthreads();
  // the lane groups of k_backsolve (2^lg lanes per column, per level) and
  // its summation order; records one level ahead; factor and x in LDS
  const int32_t* bsp = d.bs_ptr + sm.bs_ptr;
  const int32_t* bsg = d.bs_lg + sm.bs_ptr;
  const int4 none = make_int4(0, 0, 0, 0);
  int b0 = 0, b1 = 0, lg = 0;
  int4 bpre = none;
  int2 upre = make_int2(0, 0);
  if (sm.nlev > 0) {
    b0 = bsp[sm.nlev - 1];
    b1 = bsp[sm.nlev];
    lg = bsg[sm.nlev - 1];
    if (b0 + (tid >> lg) < b1) bpre = d.bs_items[b0 + (tid >> lg)];
    if (bpre.z + (tid & ((1 << lg) - 1)) < bpre.w) upre = d.bs_con[bpre.z + (tid & ((1 << lg) - 1))];
  }
  for (int lev = sm.nlev - 1; lev >= 0; --lev) {
    const int G = 1 << lg, grp = tid >> lg, gl = tid & (G - 1);
    const int nb0 = lev > 0 ? bsp[lev - 1] : b0;
    const int nlg = lev > 0 ? bsg[lev - 1] : 0;
    int4 bnext = none;
    if (lev > 0 && nb0 + (tid >> nlg) < b0) bnext = d.bs_items[nb0 + (tid >> nlg)];
    for (int it = b0 + grp; it < b1; it += NT >> lg) {
      const bool first = it == b0 + grp;
      const int4 b = first ? bpre : d.bs_items[it];
      double t0 = 0.0, t1 = 0.0;
      for (int c = b.z + gl; c < b.w; c += G) {
        const int2 u = (first && c == b.z + gl) ? upre : d.bs_con[c];
        const double* Lb = L + u.x;
        const double x0 = xl[u.y], x1 = xl[u.y + 1];
        t0 += Lb[0] * x0 + Lb[1] * x1;
        t1 += Lb[2] * x0 + Lb[3] * x1;
      }
      for (int off = G >> 1; off > 0; off >>= 1) {
        t0 += __shfl_xor(t0, off);
        t1 += __shfl_xor(t1, off);
      }
      if (gl == 0) {
        t0 = xl[b.y] - t0;
        t1 = xl[b.y + 1] - t1;
        const double* D = L + b.x;
        double l00, l10, l11, i00, i11;
        if (!chol2(D[0], D[1], D[3], l00, l10, l11, i00, i11)) {
          l00 = l11 = i00 = i11 = 1.0;
          l10 = 0.0;
        }
        const double x1 = t1 * i11;
        xl[b.y + 1] = x1;
        xl[b.y] = (t0 - l10 * x1) * i00;
      }
    }
    int2 unext = make_int2(0, 0);
    if (bnext.z + (tid & ((1 << nlg) - 1)) < bnext.w) unext = d.bs_con[bnext.z + (tid & ((1 << nlg) - 1))];
    lds_barrier();
    b1 = b0;
    b0 = nb0;
    lg = nlg;
    bpre = bnext;
    upre = unext;
  }
  for (int i = tid; i < 2 * sm.nn; i += NT) rhs[i] = xl[i];
}

// ---------------------------------------------------------------------------
// Stage 4b: x += dx for every bus, max |dx| per snapshot, convergence.
// One workgroup per snapshot.  A snapshot whose factorisation hit a
// non-positive pivot is frozen without an update.
// ---------------------------------------------------------------------------
// local != 0: a local step (boundary fixed): boundary buses, whose dx lives in
// the boundary system, do not move, and the convergence state is left alone.
__global__ void __launch_bounds__(512) k_update(Dev d, int s0, int local) {
  const int s = s0 + blockIdx.x;
  __shared__ double red[16];
  __shared__ int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (!d.active[s]) {
    if (tid == 0 && !local) d.maxdx[s] = 0.0;
    return;
  }
  const int gamma_rhs = d.sys[d.n_area].rhs_off;
  if (tid == 0) {
    int b = 0;
    for (int k = 0; k <= d.n_area; ++k) b |= d.status[(int64_t)s * (d.n_area + 1) + k];
    bad = b;
  }
  __syncthreads();
  double m = 0.0;
  if (!bad) {
    const double* rb = d.rhs + (int64_t)s * d.rstride;
    double2* xs = d.x + (int64_t)s * d.n_bus;
    for (int bus = tid; bus < d.n_bus; bus += nt) {
      const int src = d.bus_dx_src[bus];
      const bool hold = local && src >= gamma_rhs;
      const double dt = (bus == d.slack || hold) ? 0.0 : rb[src];
      const double dv = hold ? 0.0 : rb[src + 1];
      double2 v = xs[bus];
      v.x += dt;
      v.y += dv;
      xs[bus] = v;
      m = nanmax(m, fabs(dt));
      m = nanmax(m, fabs(dv));
    }
  }
  const double mx = block_max(m, red);
  if (tid == 0 && !local) {
    d.maxdx[s] = mx;
    d.iters[s] += 1;
    if (bad || mx < d.tol[0]) d.active[s] = 0;
  }
}

// (|V|, theta) arrays <-> interleaved state; flat start when vm == nullptr.
__global__ void k_pack_state(Dev d, const double* vm, const double* va, double2* xout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)d.n_snap * d.n_bus;
  if (i >= n) return;
  const int bus = (int)(i % d.n_bus);
  double2 v;
  v.x = (vm == nullptr || bus == d.slack) ? 0.0 : va[i];
  v.y = (vm == nullptr) ? 1.0 : vm[i];
  xout[i] = v;
}

__global__ void k_unpack_state(Dev d, double* vm, double* va) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)d.n_snap * d.n_bus;
  if (i >= n) return;
  const double2 v = d.x[i];
  vm[i] = v.y;
  va[i] = v.x;
}

__global__ void k_reset_flags(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.n_snap) {
    d.active[i] = 1;
    d.iters[i] = 0;
    d.maxdx[i] = 0.0;
  }
  if (i < d.n_snap * (d.n_area + 1)) d.status[i] = 0;
}

// ---------------------------------------------------------------------------
// Continuous batching over a stream of snapshots
// ---------------------------------------------------------------------------
// One workgroup of 256 threads. A slot wants work when it is idle
// (slot_id < 0) or its snapshot has finished: converged (frozen with no bad
// pivot), failed (a non-positive pivot), or out of iterations. A finished
// snapshot records its iteration count and outcome (1 converged, 0 not,
// 2 non-positive pivot); the slots that want work take the next snapshots of
// the stream in slot order (a prefix count, so the assignment is
// deterministic) and start them with cleared flags, or go idle once the
// stream is exhausted. retire[s] / refill[s] tell k_stream_copy which
// snapshot leaves and which enters slot s (-1: none). next[0] is the stream
// position; next[1] receives the lowest stream position still in a slot
// (next[0] when every slot is idle): every earlier snapshot has left.
// host_active / host_pos: device addresses of pinned host buffers that
// receive the slots' active flags and next[0..1] after the hand-over (so the
// host reads them without a copy), or null.
__global__ void __launch_bounds__(256) k_stream_refill(Dev d, int32_t* slot_id, int32_t* next,
                                                       int32_t* retire, int32_t* refill, int32_t* out_iters,
                                                       int32_t* out_flag, int32_t n_total, int32_t max_iter,
                                                       int32_t* host_active, int32_t* host_pos) {
  __shared__ int cnt[4];
  __shared__ int base;
  __shared__ int lows[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K1 = d.n_area + 1;
  int low = 0x7fffffff;
  if (tid == 0) base = *next;
  __syncthreads();
  for (int c0 = 0; c0 < d.n_snap; c0 += 256) {
    const int s = c0 + tid;
    int want = 0, leaving = -1, keep = -1, fin = 1;
    if (s < d.n_snap) {
      const int id = slot_id[s];
      keep = id;
      if (id < 0) {
        want = 1;
      } else {
        int bad = 0;
        // the pivot flags, 8 loads in flight
        for (int k0 = 0; k0 < K1; k0 += 8) {
          int f[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) f[u] = (k0 + u < K1) ? d.status[(int64_t)s * K1 + k0 + u] : 0;
#pragma unroll
          for (int u = 0; u < 8; ++u) bad |= f[u];
        }
        const int act = d.active[s];
        if (!act || bad || d.iters[s] >= max_iter) {
          want = 1;
          leaving = id;
          out_iters[id] = d.iters[s];
          out_flag[id] = bad ? 2 : (act ? 0 : 1);
        }
      }
    }
    const unsigned long long m = __ballot(want);
    if (lane == 0) cnt[wv] = __popcll(m);
    __syncthreads();
    int rank = base + __popcll(m & ((1ull << lane) - 1ull));
    for (int w = 0; w < wv; ++w) rank += cnt[w];
    if (s < d.n_snap) {
      retire[s] = leaving;
      int entering = -1;
      if (want) {
        const bool take = rank < n_total;
        entering = take ? rank : -1;
        keep = entering;
        slot_id[s] = entering;
        fin = take ? 1 : 0;
        d.active[s] = fin;
        d.iters[s] = 0;
        d.maxdx[s] = 0.0;
        for (int k = 0; k < K1; ++k) d.status[(int64_t)s * K1 + k] = 0;
      }
      refill[s] = entering;
      if (host_active) host_active[s] = fin;
      if (keep >= 0 && keep < low) low = keep;
    }
    __syncthreads();
    if (tid == 0) base += cnt[0] + cnt[1] + cnt[2] + cnt[3];
    __syncthreads();
  }
  for (int off = 32; off > 0; off >>= 1) low = min(low, __shfl_down(low, off, 64));
  if (lane == 0) lows[wv] = low;
  __syncthreads();
  if (tid == 0) {
    const int nx = base < n_total ? base : n_total;
    const int lo = min(min(lows[0], lows[1]), min(lows[2], lows[3]));
    next[0] = nx;
    next[1] = lo < nx ? lo : nx;
    if (host_pos) {
      host_pos[0] = nx;
      host_pos[1] = lo < nx ? lo : nx;
    }
  }
}

// Every slot idle and the stream position at 0 (a kernel rather than a
// memset, so that the clearing also behaves inside captured work).
__global__ void k_stream_init(int32_t* slot_id, int32_t* next, int n_snap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_snap) slot_id[i] = -1;
  if (i < 2) next[i] = 0;
}

constexpr int STREAM_COPY_CHUNKS = 32;  // workgroups per slot

// Grid (chunks, n_snap). Slot s hands the state of its finished snapshot to
// vm_out / va_out [n_total][n_bus] and loads the entering snapshot's
// measurements (zs [n_total][n_meas]) and starting state (vm0 / va0
// [n_total][n_bus], flat start when vm0 is null; slack angle 0).
__global__ void k_stream_copy(Dev d, const int32_t* retire, const int32_t* refill, const double* zs,
                              const double* vm0, const double* va0, double* vm_out, double* va_out) {
  const int s = blockIdx.y;
  const int leaving = retire[s], entering = refill[s];
  if (leaving < 0 && entering < 0) return;
  const int stride = gridDim.x * blockDim.x;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  double2* xs = d.x + (int64_t)s * d.n_bus;
  for (int i = i0; i < d.n_bus; i += stride) {
    double2 v = xs[i];
    if (leaving >= 0) {
      vm_out[(int64_t)leaving * d.n_bus + i] = v.y;
      va_out[(int64_t)leaving * d.n_bus + i] = v.x;
    }
    if (entering >= 0) {
      const int64_t e = (int64_t)entering * d.n_bus + i;
      v.x = (vm0 == nullptr || i == d.slack) ? 0.0 : va0[e];
      v.y = vm0 == nullptr ? 1.0 : vm0[e];
      xs[i] = v;
    }
  }
  if (entering >= 0) {
    // U measurements per thread and pass, loaded together
    constexpr int U = 4;
    const double* src = zs + (int64_t)entering * d.n_meas;
    double* dst = const_cast<double*>(d.z) + (int64_t)s * d.n_meas;
    for (int j0 = i0; j0 < d.n_meas; j0 += U * stride) {
      double t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) t[u] = (j0 + u * stride < d.n_meas) ? src[j0 + u * stride] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (j0 + u * stride < d.n_meas) dst[j0 + u * stride] = t[u];
    }
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
constexpr int AREA_NT = 256;   // level kernels over areas: many workgroups
constexpr size_t BACKSOLVE_LDS_MAX = 65536;  // rhs staged in LDS up to 4096 buses per system
constexpr size_t ELIM_LDS_MAX = 65536;       // elimination staging + rhs in LDS up to this size
constexpr int GAMMA_NT = 1024; // level kernels over the one boundary system

size_t assemble_lds_bytes(int nn, int nbr, bool br_lds, int nrow) {
  return 16 * (size_t)nn + 16 * (size_t)nbr + 48 * (size_t)nn + (br_lds ? sizeof(BrL) * (size_t)nbr : 0) +
         16 * (size_t)nrow;
}

hipError_t launch_assemble(const Dev& d, int a0, int na, int s0, int ns, int mode, size_t lds,
                           bool br_lds, hipStream_t st) {
  if (na <= 0 || ns <= 0) return hipSuccess;
  if (d.asm_stage)
    hipLaunchKernelGGL((k_assemble<false, true, false>), dim3(na * ns), dim3(ASM_NT), 0, st, d, a0, na, s0, ns,
                       mode);
  else if (br_lds && d.asm_wz)
    hipLaunchKernelGGL((k_assemble<true, false, true>), dim3(na * ns), dim3(ASM_NT), lds, st, d, a0, na, s0, ns,
                       mode);
  else if (br_lds)
    hipLaunchKernelGGL((k_assemble<true, false, false>), dim3(na * ns), dim3(ASM_NT), lds, st, d, a0, na, s0, ns,
                       mode);
  else if (d.asm_wz)
    hipLaunchKernelGGL((k_assemble<false, false, true>), dim3(na * ns), dim3(ASM_NT), lds, st, d, a0, na, s0, ns,
                       mode);
  else
    hipLaunchKernelGGL((k_assemble<false, false, false>), dim3(na * ns), dim3(ASM_NT), lds, st, d, a0, na, s0, ns,
                       mode);
  return hipGetLastError();
}

hipError_t launch_eliminate(const Dev& d, int sys0, int nsys, int s0, int ns, size_t lds, hipStream_t st) {
  if (nsys <= 0 || ns <= 0) return hipSuccess;
  // LDS: the staging area (lds bytes), then the largest system's rhs when
  // the two fit in ELIM_LDS_MAX
  const int lstride = (int)(lds / sizeof(double));
  const bool gamma = sys0 >= d.n_area;
  const size_t rl = 16 * (size_t)(gamma ? d.bs_max_nn_gamma : d.bs_max_nn_area);
  const bool in_lds = lds + rl <= ELIM_LDS_MAX;
  const size_t bytes = in_lds ? lds + rl : lds;
  const dim3 grid(nsys * ns);
  if (gamma) {
    if (in_lds)
      hipLaunchKernelGGL((k_eliminate<GAMMA_NT, true>), grid, dim3(GAMMA_NT), bytes, st, d, sys0, nsys, s0, ns, lstride);
    else
      hipLaunchKernelGGL((k_eliminate<GAMMA_NT, false>), grid, dim3(GAMMA_NT), bytes, st, d, sys0, nsys, s0, ns, lstride);
  } else {
    if (in_lds)
      hipLaunchKernelGGL((k_eliminate<AREA_NT, true>), grid, dim3(AREA_NT), bytes, st, d, sys0, nsys, s0, ns, lstride);
    else
      hipLaunchKernelGGL((k_eliminate<AREA_NT, false>), grid, dim3(AREA_NT), bytes, st, d, sys0, nsys, s0, ns, lstride);
  }
  return hipGetLastError();
}

hipError_t launch_elim_lds(const Dev& d, int a0, int na, int s0, int ns, size_t lds, int nt, bool tail_hbm,
                           hipStream_t st) {
  if (na <= 0 || ns <= 0) return hipSuccess;
  const dim3 grid(na * ns);
#define ELIM_LDS_CASE(N)                                                                              \
  if (nt == N) {                                                                                      \
    if (tail_hbm)                                                                                     \
      hipLaunchKernelGGL((k_elim_lds<N, true>), grid, dim3(N), lds, st, d, a0, na, s0, ns);           \
    else                                                                                              \
      hipLaunchKernelGGL((k_elim_lds<N, false>), grid, dim3(N), lds, st, d, a0, na, s0, ns);          \
    return hipGetLastError();                                                                         \
  }
  ELIM_LDS_CASE(256)
  ELIM_LDS_CASE(512)
  ELIM_LDS_CASE(1024)
#undef ELIM_LDS_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_back_lds(const Dev& d, int a0, int na, int s0, int ns, size_t lds, int nt, bool fixed_bnd,
                           hipStream_t st) {
  if (na <= 0 || ns <= 0) return hipSuccess;
  const dim3 grid(na * ns);
  const int fb = fixed_bnd ? 1 : 0;
  if (nt == 256) hipLaunchKernelGGL((k_back_lds<256>), grid, dim3(256), lds, st, d, a0, na, s0, ns, fb);
  else if (nt == 512) hipLaunchKernelGGL((k_back_lds<512>), grid, dim3(512), lds, st, d, a0, na, s0, ns, fb);
  else if (nt == 1024) hipLaunchKernelGGL((k_back_lds<1024>), grid, dim3(1024), lds, st, d, a0, na, s0, ns, fb);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t allow_elim_lds(size_t bytes) {
  const void* g[3] = {reinterpret_cast<const void*>(&k_back_lds<256>),
                      reinterpret_cast<const void*>(&k_back_lds<512>),
                      reinterpret_cast<const void*>(&k_back_lds<1024>)};
  for (const void* fn : g) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  const void* f[6] = {reinterpret_cast<const void*>(&k_elim_lds<256, false>),
                      reinterpret_cast<const void*>(&k_elim_lds<256, true>),
                      reinterpret_cast<const void*>(&k_elim_lds<512, false>),
                      reinterpret_cast<const void*>(&k_elim_lds<512, true>),
                      reinterpret_cast<const void*>(&k_elim_lds<1024, false>),
                      reinterpret_cast<const void*>(&k_elim_lds<1024, true>)};
  for (const void* fn : f) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t allow_eliminate_lds(size_t bytes) {
  const void* f[4] = {reinterpret_cast<const void*>(&k_eliminate<GAMMA_NT, true>),
                      reinterpret_cast<const void*>(&k_eliminate<GAMMA_NT, false>),
                      reinterpret_cast<const void*>(&k_eliminate<AREA_NT, true>),
                      reinterpret_cast<const void*>(&k_eliminate<AREA_NT, false>)};
  for (const void* fn : f) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gamma_gather(const Dev& d, int s0, int ns, int nslot, int nn, hipStream_t st) {
  const int work = nslot > nn ? nslot : nn;
  if (work <= 0 || ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gamma_gather, dim3((work + 255) / 256, ns), dim3(256), 0, st, d, s0, nslot);
  return hipGetLastError();
}

hipError_t launch_gamma_snode(const Dev& d, int s0, int ns, size_t lds, hipStream_t st) {
  if (ns <= 0 || d.n_sn <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gamma_snode, dim3(ns * d.n_sn_grp), dim3(SN_NT), lds, st, d, s0);
  if (d.n_tail_ent > 0) {
    const int nblk = (d.n_tail_ent + TAIL_NT - 1) / TAIL_NT;
    hipLaunchKernelGGL(k_gamma_tail, dim3(ns * nblk), dim3(TAIL_NT), 0, st, d, s0, nblk);
  }
  return hipGetLastError();
}

hipError_t allow_gamma_snode_lds(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gamma_snode),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

size_t dense_lds_bytes(int ld, int mode, int nb) {
  if (mode == DENSE_WIDE) return sizeof(double) * ((size_t)ld + (size_t)nb * (ld + 1));
  return sizeof(double) * ((size_t)ld + (mode == DENSE_PANEL16 ? (size_t)ld * PANEL_PITCH : 0));
}

hipError_t launch_dense_chol(const Dev& d, int s0, int ns, int ld, int mode, int nb, hipStream_t st) {
  if (ld <= 0 || ns <= 0) return hipSuccess;
  const size_t lds = dense_lds_bytes(ld, mode, nb);
  if (mode == DENSE_WIDE)
    hipLaunchKernelGGL(k_dense_wide, dim3(ns), dim3(DW_NT), lds, st, d, s0, nb);
  else if (mode == DENSE_PANEL16)
    hipLaunchKernelGGL(k_dense_chol<true>, dim3(ns), dim3(DENSE_NT), lds, st, d, s0);
  else
    hipLaunchKernelGGL(k_dense_chol<false>, dim3(ns), dim3(DENSE_NT), lds, st, d, s0);
  return hipGetLastError();
}

hipError_t allow_dense_lds(int mode, size_t bytes) {
  const void* f = mode == DENSE_WIDE ? reinterpret_cast<const void*>(&k_dense_wide)
                                     : reinterpret_cast<const void*>(&k_dense_chol<true>);
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_backsolve(const Dev& d, int sys0, int nsys, int s0, int ns, hipStream_t st, bool fixed_bnd) {
  if (nsys <= 0 || ns <= 0) return hipSuccess;
  // LDS: the largest system's rhs (2 doubles per local bus), if it fits
  if (sys0 >= d.n_area) {
    const size_t lds = 16 * (size_t)d.bs_max_nn_gamma;
    if (lds <= BACKSOLVE_LDS_MAX)
      hipLaunchKernelGGL((k_backsolve<GAMMA_NT, true>), dim3(nsys * ns), dim3(GAMMA_NT), lds, st, d, sys0, nsys, s0,
                         ns, 0);
    else
      hipLaunchKernelGGL((k_backsolve<GAMMA_NT, false>), dim3(nsys * ns), dim3(GAMMA_NT), 0, st, d, sys0, nsys, s0,
                         ns, 0);
  } else {
    const size_t lds = 16 * (size_t)d.bs_max_nn_area;
    if (lds <= BACKSOLVE_LDS_MAX)
      hipLaunchKernelGGL((k_backsolve<AREA_NT, true>), dim3(nsys * ns), dim3(AREA_NT), lds, st, d, sys0, nsys, s0,
                         ns, fixed_bnd ? 1 : 0);
    else
      hipLaunchKernelGGL((k_backsolve<AREA_NT, false>), dim3(nsys * ns), dim3(AREA_NT), 0, st, d, sys0, nsys, s0,
                         ns, fixed_bnd ? 1 : 0);
  }
  return hipGetLastError();
}

hipError_t launch_update(const Dev& d, int s0, int ns, hipStream_t st, bool local) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update, dim3(ns), dim3(512), 0, st, d, s0, local ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_pack_state(const Dev& d, const double* vm, const double* va, double2* xout,
                             hipStream_t st) {
  const int64_t n = (int64_t)d.n_snap * d.n_bus;
  hipLaunchKernelGGL(k_pack_state, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, vm, va, xout);
  return hipGetLastError();
}

hipError_t launch_unpack_state(const Dev& d, double* vm, double* va, hipStream_t st) {
  const int64_t n = (int64_t)d.n_snap * d.n_bus;
  hipLaunchKernelGGL(k_unpack_state, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, vm, va);
  return hipGetLastError();
}

hipError_t launch_reset_flags(const Dev& d, hipStream_t st) {
  const int n = d.n_snap * (d.n_area + 1);
  hipLaunchKernelGGL(k_reset_flags, dim3((n + 255) / 256), dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_stream_refill(const Dev& d, int32_t* slot_id, int32_t* next, int32_t* retire,
                                int32_t* refill, int32_t* out_iters, int32_t* out_flag, int32_t n_total,
                                int32_t max_iter, int32_t* host_active, int32_t* host_pos, hipStream_t st) {
  hipLaunchKernelGGL(k_stream_refill, dim3(1), dim3(256), 0, st, d, slot_id, next, retire, refill, out_iters,
                     out_flag, n_total, max_iter, host_active, host_pos);
  return hipGetLastError();
}

hipError_t launch_stream_init(int32_t* slot_id, int32_t* next, int n_snap, hipStream_t st) {
  const int n = n_snap > 2 ? n_snap : 2;
  hipLaunchKernelGGL(k_stream_init, dim3((n + 255) / 256), dim3(256), 0, st, slot_id, next, n_snap);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const Dev& d, const int32_t* retire, const int32_t* refill, const double* zs,
                              const double* vm0, const double* va0, double* vm_out, double* va_out,
                              hipStream_t st) {
  // STREAM_COPY_CHUNKS workgroups of 256 threads per slot cover the measurement
  // copy (the larger part) with few passes each
  hipLaunchKernelGGL(k_stream_copy, dim3(STREAM_COPY_CHUNKS, (unsigned)d.n_snap), dim3(256), 0, st, d, retire,
                     refill, zs, vm0, va0, vm_out, va_out);
  return hipGetLastError();
}

hipError_t allow_assemble_lds(size_t bytes, bool br_lds) {
  const void* f[2] = {br_lds ? reinterpret_cast<const void*>(&k_assemble<true, false, true>)
                             : reinterpret_cast<const void*>(&k_assemble<false, false, true>),
                      br_lds ? reinterpret_cast<const void*>(&k_assemble<true, false, false>)
                             : reinterpret_cast<const void*>(&k_assemble<false, false, false>)};
  for (const void* fn : f) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mase
