// Device kernels of the FR right-hand side and their host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace fr {

// ----------------------------------------------------------------------------
// Operator GEMM  C = A [B1; B2]  (Appendix A form C <- A B), A packed on the
// host into MFMA fragment order.  Columns are the SoA state columns
// alpha*ld + n; rows are solution/flux points (times spatial components).
// ----------------------------------------------------------------------------
enum GemmEpi {
  EPI_STORE = 0,   // C[row][col] = acc                         (C of type TC)
  EPI_NEGDIV = 1,  // out = -rcpdjac[row][n] * acc, 0 for padding  (FP64 out)
  EPI_RK = 2,      // RK4 stage update from k = -rcpdjac * acc      (FP64 regs)
  EPI_ADD = 3,     // C[row][col] += acc (FP64 only; adjoint accumulation)
  EPI_GRADT = 4,   // sparse-row kernel only: the D rows d Nu + rho of one point
                   // are transformed by J^-T = S^T / det J before the store
  EPI_ADDT = 5,    // sparse-row kernel only (adjoint, FP64): row rho of the D
                   // batch slices is added to C, then the D sums of one point
                   // are transformed by J^-1 = S / det J (the reverse of the
                   // gradient transform); padding columns are only added
  EPI_GRADTF = 6,  // sparse-row kernel, every field of an element per thread
                   // (Navier-Stokes): EPI_GRADT, then the transformed flux
                   // F~ = S f(u, Q) of the point from the stored Q and the
                   // state (panel 2) into fout; padding columns get 0
  EPI_RKADJ = 8,   // sparse-row kernel (adjoint, FP64): w = C + acc is the
                   // state cotangent of an RK stage; then the step adjoint's
                   // bookkeeping: acc_reg += w and (unless rk.last) out =
                   // -rcpdjac (rk.a_next dt lam + rk.b dt w), lam read from
                   // `stage`; C is only read; padding columns of out get 0
  EPI_TFVJP = 7    // sparse-row kernel, every field of an element per thread
                   // (adjoint, FP64): the D rows d Nu + rho of one point are
                   // F~b; then fb = S^T F~b and the reverse of the flux,
                   // ub = (df/du)^T fb into `out` (the state cotangent) and,
                   // with a primal Q (qprim), qb = (df/dq)^T fb into C;
                   // padding columns get 0
};

enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };

struct RkCoef {
  double a_next;    // stage_next = u + a_next * dt * k  (ignored on the last stage)
  double b;         // acc += b * dt * k
  int first;        // acc is initialised from u on the first stage
  int last;         // u = acc + b dt k on the last stage (no stage write)
};

struct GemmArgs {
  const void *Apack;      // packed operator (precision dependent element type)
  int M;                  // rows of A (= rows of C)
  int KS1, KS2;           // k-steps (of the MFMA K) in each panel
  int K1, K2;             // true K of each panel
  int MBW;                // row blocks (16 rows) per wave
  int NC;                 // 16-column strips per wave
  int WM;                 // waves along M sharing one column tile
  const void *B1; int64_t ldb1; int b1_f32;   // panel 1 (rows K1), row stride
  const void *B2; int64_t ldb2; int b2_f32;   // panel 2 (rows K2)
  void *C; int64_t ldc; int c_f32;            // output (EPI_STORE)
  int64_t N;              // columns (nvars * ld)
  int64_t sB1, sC;        // batch strides (blockIdx.y) in elements
  // epilogue data
  const double *rcpdjac; int64_t ld; int64_t nelem;
  double *out;            // EPI_NEGDIV output / EPI_RK: u (in/out)
  double *acc; double *stage;
  const double *dt; const int32_t *prob;      // per-problem step size, element -> problem
  RkCoef rk;
  const double *smat; int D; int Nu;          // EPI_GRADT: S = adj J [D][D][Nu][ld]
  void *fout; double gamma, mu, prandtl;      // EPI_GRADTF: F~ (type TC, layout of C)
  // EPI_TFVJP: primal u and Q (Q null: Euler); EPI_GRADTF: u (the FP64
  // state, rows of ldb values), with devflux: F~ less S f(u_ref), u_ref the
  // element's first solution point (deviation form)
  const double *uprim, *qprim;
  int devflux;
  // sparse-row kernel with precomputed gathers: roff[r * width + e] is the
  // byte offset, from rbase, of the B row of entry e of operator row r
  // (both panels), rbase + (batch slice) addressed through one 32-bit
  // buffer range; null: rows located from the column index at run time
  const uint32_t *roff; const void *rbase;
  // multi-block launch: one launch covers the workgroups of every slot; the
  // pointers above are then the bases of whole arrays (slot offsets added)
  const struct LaunchSlot *slots; int nslots; int64_t nwg;  // nwg: workgroups of all slots
};

// One element block of a multi-block launch (one launch of an operator
// product over several blocks of a mixed or batched mesh): its workgroups
// [wg_begin, next slot's wg_begin), the element offsets of its operands
// from the launch's base pointers, and its own operator and geometry.
struct LaunchSlot {
  int64_t wg_begin;
  int64_t off_b1, off_b2, off_c, off_u;   // B1, B2, C, and out/acc/stage
  int64_t ld, N, nelem, sB1, sC;           // ldb1 = ldb2 = ldc = N
  const void *Apack;                       // matrix-core plans
  const int32_t *colidx; const double *vals; const uint32_t *roff;  // sparse-row plans
  int rbase_b2;                            // two panels: rbase is B2 (else B1)
  const double *rcpdjac; const int32_t *prob;
  int M, K1, K2, KS1, KS2, WM, rpg, ngroups;
};

// Patch a multi-block launch's arguments with the slot of workgroup `wg`
// (slots sorted by wg_begin, at most a few dozen); returns the workgroup's
// index within its slot.  Element sizes: ts1 (B1), ts2 (B2), tc (C).
__device__ __forceinline__ int64_t take_slot(GemmArgs &g, int64_t wg, size_t ts1, size_t ts2,
                                             size_t tc, const LaunchSlot **which = nullptr) {
  int k = 0;
  while (k + 1 < g.nslots && wg >= g.slots[k + 1].wg_begin) ++k;
  const LaunchSlot &sl = g.slots[k];
  if (which) *which = &sl;
  g.B1 = (const char *)g.B1 + sl.off_b1 * (int64_t)ts1;
  if (g.B2) g.B2 = (const char *)g.B2 + sl.off_b2 * (int64_t)ts2;
  if (g.C) g.C = (char *)g.C + sl.off_c * (int64_t)tc;
  if (g.out) g.out += sl.off_u;
  if (g.acc) g.acc += sl.off_u;
  if (g.stage) g.stage += sl.off_u;
  g.ldb1 = g.ldb2 = g.ldc = g.N = sl.N;
  g.ld = sl.ld; g.nelem = sl.nelem; g.sB1 = sl.sB1; g.sC = sl.sC;
  g.Apack = sl.Apack; g.roff = sl.roff;
  g.rbase = sl.rbase_b2 ? g.B2 : g.B1;
  g.rcpdjac = sl.rcpdjac; g.prob = sl.prob;
  g.M = sl.M; g.K1 = sl.K1; g.K2 = sl.K2; g.KS1 = sl.KS1; g.KS2 = sl.KS2; g.WM = sl.WM;
  return wg - sl.wg_begin;
}

// Pack A (M x (K1 + K2), row-major, panel 2 columns follow panel 1) into the
// fragment layout the kernel reads; returns element count, writes into dst
// (may be null to query).  kstep = 4 for FP64/FP32.
int64_t gemm_pack_size(int M, int K1, int K2, int MBW, int WM, int kstep);
void gemm_pack_f64(const double *A, int M, int K1, int K2, int MBW, int WM, double *dst);
void gemm_pack_f32(const double *A, int M, int K1, int K2, int MBW, int WM, float *dst);
// BF16x3: k-steps of 32; hi and lo bf16 fragments interleaved (see kernel)
int64_t gemm_pack_size_bf16(int M, int K1, int K2, int MBW, int WM);
void gemm_pack_bf16x3(const double *A, int M, int K1, int K2, int MBW, int WM, uint16_t *dst);

hipError_t launch_gemm(int prec, int epi, const GemmArgs &g, int batch, hipStream_t s);
hipError_t launch_gemm_f64(int epi, const GemmArgs &g, int batch, hipStream_t s);
hipError_t launch_gemm_f32(int epi, const GemmArgs &g, int batch, hipStream_t s);
hipError_t launch_gemm_bf16x3(int epi, const GemmArgs &g, int batch, hipStream_t s);

// Operator stored with a fixed number of entries per row (ELL) for the
// sparse-row kernel (spop.hip): row r holds colidx[r * width + e] and
// vals[r * width + e], e < width; padding entries have value 0.
struct SparseOp {
  const int32_t *colidx;   // [M][width], column in [0, K1 + K2)
  const double *vals;      // [M][width]
  int width;               // one of FR_SPOP_WIDTHS
  int rpg;                 // operator rows per workgroup row
  int fields;              // fields per thread: 1, or the field count (N = fields * ld)
  // precomputed byte offsets of every entry's B row ([M][width]) for the
  // operand arrays of the context's own right-hand side: from panel 1 for a
  // one-panel operator (valid for any operand address), from the lower of
  // the two panels otherwise (valid while B2 - B1 == roff_delta bytes)
  const uint32_t *roff = nullptr;
  int64_t roff_delta = 0;
};
#define FR_SPOP_WIDTHS(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(14) X(15) X(16) X(18) X(20) X(21) X(24) X(32)
// the fused gradient transform with every field in one thread holds D x N_V
// accumulators besides the row's loads: instantiated up to this width only
#define FR_SPOP_GRADT_FIELDS_WMAX 16
// smallest instantiated width >= nnz_max (0 if none)
int spop_width(int nnz_max);

// LDS-staged form of a sparse operator (spop_lds.h).  The K = K1 + K2 rows
// of B are taken in chunks of kc rows; chunk c holds, for every operator row
// r, colidx[(c M + r) width + e] (a row of B within the chunk) and
// vals[...], e < width; padding entries have value 0.
struct StagedOp {
  const int32_t *colidx;   // [nchunk][M][width]
  const double *vals;      // [nchunk][M][width]
  int width;               // one of FR_LDS_WIDTHS (at least every chunk's own width)
  int kc;                  // most B rows of a chunk (kc x 64 values of LDS)
  int nchunk;
  // chunk c holds B rows [cstart[c], cstart[c + 1]); its rows hold cwidth[c]
  // entries each (the rest of `width` unused).  Chunks follow the operator's
  // structure where they can (the faces of a face group, one direction of the
  // transformed flux), so every row of a chunk has about the same count.
  const int32_t *cstart = nullptr;
  const int32_t *cwidth = nullptr;
};
#define FR_LDS_WIDTHS(X) X(4) X(5) X(6) X(8) X(12)
// most B rows of one LDS chunk, in every precision (32 per wavefront)
constexpr int kStagedRows = 128;
// output rows per wavefront (4 wavefronts split the M rows of a tile)
#define FR_LDS_ROWS(X) X(4) X(8) X(16) X(24) X(32) X(40)
#define FR_LDS_ROWS_MAX 40
// the fused gradient transform keeps D accumulators per point
#define FR_LDS_GRADT_ROWS_MAX 16
hipError_t launch_spop_lds(int prec, int epi, const GemmArgs &g, const StagedOp &op, int batch,
                           hipStream_t s);
hipError_t launch_spop_lds_f64(int epi, const GemmArgs &g, const StagedOp &op, int batch,
                               hipStream_t s);
hipError_t launch_spop_lds_f32(int epi, const GemmArgs &g, const StagedOp &op, int batch,
                               hipStream_t s);
// smallest instantiated chunk width >= nnz_max (0 if none)
int spop_lds_width(int nnz_max);
hipError_t launch_spop(int prec, int epi, const GemmArgs &g, const SparseOp &sp, int batch,
                       hipStream_t s);
// One launch over every slot of g.slots (g.nwg workgroups): the sparse-row
// kernel with precomputed gathers, ELL width `width` in every slot, `fields`
// fields per thread; epilogues store, -1/J and RK.
hipError_t launch_spop_multi(int prec, int epi, const GemmArgs &g, int width, int fields,
                             int batch, hipStream_t s);
hipError_t launch_spop_multi_fields(int prec, int epi, const GemmArgs &g, int width, int fields,
                                    int batch, hipStream_t s);
// workgroups (four wavefronts each) of one block's matrix-core launch
inline int64_t gemm_workgroups(int64_t N, int NC, int WM) {
  return ((N + 16 * NC - 1) / (16 * NC) * WM + 3) / 4;
}
// workgroups of one block's sparse-row launch (column tiles padded to a
// multiple of the 8 XCDs, times the row groups)
inline int64_t spop_workgroups(int64_t threads, int M, int rpg) {
  return ((threads + 255) / 256 + 7) / 8 * 8 * ((M + rpg - 1) / rpg);
}

// LDS-staged BF16x3 plans (MBW, WM, column tile TW = NC): four wavefronts
// per workgroup split WM row groups and TW / 16 strips
#define FR_BF16_LDS_SHAPES(X)                                                                 \
  X(1, 4, 64) X(2, 4, 64) X(3, 4, 64) X(4, 4, 64) X(6, 4, 64)                                \
  X(1, 2, 64) X(2, 2, 64) X(3, 2, 64) X(4, 2, 64) X(6, 2, 64) X(8, 2, 64)                    \
  X(1, 1, 64) X(2, 1, 64) X(3, 1, 64) X(4, 1, 64) X(6, 1, 64) X(8, 1, 64) X(12, 1, 64)       \
  X(1, 4, 128) X(2, 4, 128)                                                                  \
  X(1, 2, 128) X(2, 2, 128) X(3, 2, 128) X(4, 2, 128)                                        \
  X(1, 1, 128) X(2, 1, 128) X(4, 1, 128) X(6, 1, 128) X(8, 1, 128)

// MBW > 0: matrix-core plan; MBW == 0: sparse-row kernel with NC = rows per group.
struct GemmPlan { int MBW, NC, WM; };
// Default plan for an M-row operator and N columns (no tuning).
GemmPlan gemm_plan(int M, int64_t N, int prec);
// Every instantiated plan worth timing for this shape (autotuner).
std::vector<GemmPlan> gemm_candidates(int M, int64_t N, int prec);
bool gemm_plan_valid(int MBW, int NC);
// with the row split and the precision (NC >= 64: LDS-staged BF16x3 plans)
bool gemm_plan_valid(int MBW, int NC, int WM, int prec);

// ----------------------------------------------------------------------------
// Point-wise and interface kernels
// ----------------------------------------------------------------------------
struct PointArgs {
  int ndims, nvars, nupts;
  int64_t ld, nelem;
  const double *smat;      // [D][D][Nu][ld]
  const double *rcpdjac;   // [Nu][ld]
  const double *u;         // state [Nu][NV][ld]
  void *q;                 // gradients / transformed flux [D][Nu][NV][ld] (in place)
  void *fout;              // transformed-flux output (null: over q)
  int q_f32;
  double gamma, mu, prandtl;
  // multi-block launch: the pointers above are whole-array bases and each
  // slot names its block's part (nwg workgroups in all)
  const struct PointSlot *slots; int nslots; int64_t nwg;
  // Euler in reduced precision: deviation form.  udev (type of q, state
  // layout) receives u - u_ref, uref [NV][ld] receives the reference state
  // of each element (its state at solution point 0), and the transformed
  // flux is written as S (f(u) - f(u_ref)).  Null: plain form.
  void *udev; double *uref;
};

// One element block of a multi-block point-wise launch.
struct PointSlot {
  int64_t wg_begin;
  int64_t off_u, off_q;      // elements of u (and udev), and of q / fout (same layout)
  int64_t off_ref;           // elements of uref
  int nupts; int64_t ld, nelem;
  const double *smat, *rcpdjac;
};

// workgroups of one block's point-wise launch
inline int64_t point_workgroups(int nupts, int64_t ld) { return ((int64_t)nupts * ld + 255) / 256; }

// S4: q = J^-T q~ in place
hipError_t launch_gradcoru(const PointArgs &a, hipStream_t s);
// S6: f~ = S f(u, q) (Euler reads no q, writes f~ into q's storage)
hipError_t launch_tflux(const PointArgs &a, int navier_stokes, hipStream_t s);
// Deviation form (Navier-Stokes, reduced precision): a.udev = u - u_ref and
// a.uref = u_ref, the first solution point of each element (FP64).
hipError_t launch_devstate(const PointArgs &a, hipStream_t s);

struct PairArgs {
  int ndims, nvars;
  int64_t npairs;
  const int32_t *lidx, *ridx;      // within-block flux-point index sigma*NV*ld + n
  const int32_t *lblk, *rblk;      // block of each side (null: single block)
  const double *nrm;               // [D][npairs]
  const double *magL, *magR;
  void *uf; int uf_f32;            // U^f -> D~ in place
  void *dfout;                     // D~ output (null: over U^f)
  void *cf;                        // C^f output (con_u)
  const void *qf;                  // Q^f (NS common flux)
  const int64_t *blk_ufbase;       // per block: offset into uf/cf
  const int64_t *blk_qfbase;       // per block: offset into qf
  const int64_t *blk_ld;           // per block: leading dimension
  const int64_t *blk_qstride;      // per block: Nf * NV * ld
  int64_t ld0, qstride0;           // single-block values
  double gamma, mu, prandtl, beta, tau;
  // boundary flux points (launch_bc_*): npairs of them, lidx/lblk/nrm/magL
  // describe the point, bcid its boundary, bcpar[bc * FR_BC_NPAR + ...] the
  // boundary's parameters (layout of bc_ghosts in physics.h)
  const int32_t *bcid;
  const double *bcpar;
  // Euler in reduced precision (deviation form): U^f holds U^f - u_ref of
  // each side's element, uref [NV][ld] per block (blk_refbase: offsets of
  // multi-block meshes) the references; the common flux is rebuilt from
  // u_ref + U^f in FP64 and D~ written as J^f n^f (F - n.f(u_ref)).
  const double *uref;
  const int64_t *blk_refbase;
};
#define FR_BC_NPAR 12

// S2: common solution to both sides
hipError_t launch_con_u(const PairArgs &a, hipStream_t s);
// S7: common normal flux, scaled per side, in place over U^f
hipError_t launch_comm_flux(const PairArgs &a, int navier_stokes, hipStream_t s);
// S2 and S7 at boundary flux points (Appendix C ghost states)
hipError_t launch_bc_con_u(const PairArgs &a, hipStream_t s);
hipError_t launch_bc_comm_flux(const PairArgs &a, int navier_stokes, hipStream_t s);

// ----------------------------------------------------------------------------
// Reductions
// ----------------------------------------------------------------------------
// per-element integrals of (u[alpha] for alpha<NV, kinetic energy) into
// part[(chunk * (nvars + 1) + c) * pstride + n], chunk < nchunk (solution
// point ranges)
hipError_t launch_elem_integrals(int nvars, int ndims, int nupts, int64_t ld, int64_t nelem,
                                 int nchunk, int64_t pstride, const double *wdjac,
                                 const double *u, double *part, hipStream_t s);
// sum the partials per problem in fixed order: element lists in CSR form
// (pstart[nprob+1], plist), nslice workgroups of `per` list entries per
// problem (per a multiple of 64, nslice * per >= longest list), part2 holds
// nprob * nslice * ncomp slice sums when nslice > 1; ncomp is 1, 5 or 6
hipError_t launch_problem_sums(int ncomp, int nprob, int nchunk, int64_t pstride, int nslice,
                               int64_t per, const int64_t *pstart, const int64_t *plist,
                               const double *part, double *part2, double *out, hipStream_t s);
// The integrals' fixed scratch (element partials, then slice partials) for
// callers that cannot allocate: kIntegralScratchDoubles doubles (32 MiB) per
// device.  integral_scratch returns its address on the current device
// (hipGetSymbolAddress, resolved once per device).  Every call on a device
// shares that device's copy: calls that overlap on one device race.
constexpr int64_t kIntegralScratchDoubles = int64_t(1) << 22;
hipError_t integral_scratch(double **ptr);
// measured ceilings: kind 0 HBM triad GB/s, 1 FP64 MFMA TFLOP/s, 2 FP32 MFMA TFLOP/s
hipError_t measure_ceiling(int kind, double *value, hipStream_t s);
// flag[0] = 1 if any u is not finite
hipError_t launch_check_finite(const double *u, int64_t n, int32_t *flag, hipStream_t s);

}  // namespace fr
