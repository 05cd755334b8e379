// C ABI of the FR library: context set-up, the right-hand-side kernel chain,
// RK4 stepping (captured once into a HIP graph and replayed), integrals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/fr.h"
#include "adjoint.h"
#include "kernels.h"
#include "setup.h"
#include "steppers.h"

namespace {

thread_local std::string g_setup_error = "no error";

struct GemmOp {
  int M = 0, K1 = 0, K2 = 0, KS1 = 0, KS2 = 0, MBW = 1, NC = 1, WM = 1;
  void *d_A = nullptr;
  std::vector<double> A;  // unpacked operator (kept for re-packing by the tuner)
  fr::SparseOp sp{nullptr, nullptr, 0, 0, 1};  // ELL copy when the operator is sparse
  std::vector<int32_t> ell_cols;                // host copies of sp.colidx, sp.vals, sp.roff
  std::vector<double> ell_vals;
  std::vector<uint32_t> roff_host;
  int64_t roff_rs1 = 0, roff_rs2 = 0;          // row strides (bytes) sp.roff was built for
  fr::StagedOp st{nullptr, nullptr, 0, 0, 0};  // chunked ELL copy for the LDS-staged kernel
  double density = 1.0;
};

// Entries below this fraction of their row's largest magnitude are the
// rounding residue of structural zeros (the Vandermonde construction does
// not produce exact zeros); the sparse-row kernel skips them.
const double kSparseDrop = 1e-13;

// Sparse-row plans: MBW = 0, NC = operator rows per workgroup, WM = flags
// (bit 0: the gradient transform fused into step 3, bit 1: every field of
// an element in one thread, bit 2: the LDS-staged kernel, which takes all
// rows of 64 columns per workgroup and ignores NC, bit 3: with bits 0 and 1,
// the transformed flux of step 6 fused into step 3 as well).
const int kPlanFusedGradT = 1, kPlanFields = 2, kPlanStaged = 4, kPlanFusedFlux = 8;
// Adjoint (M1 - M3 M2)^T product: bit 4, with bit 1, applies the reverse of
// the transformed flux in its epilogue (the point-wise flux VJP pass goes).
const int kPlanFusedFluxVjp = 16;
const int kPlanFusedAll = kPlanFusedGradT | kPlanFields | kPlanFusedFlux;

void apply_sparse_plan(GemmOp &op, const fr::GemmPlan &p, int nvars) {
  op.sp.rpg = p.NC;
  op.sp.fields = (p.WM & kPlanFields) ? nvars : 1;
}

// Whether the LDS-staged kernel has an instantiation for this operator
// (rows per wavefront, and points per wavefront when fused with the gradient
// transform of a D-dimensional block).
bool staged_ok(const GemmOp &op, bool fused, int D) {
  if (!op.st.colidx) return false;
  if (fused) return op.M % D == 0 && (op.M / D + 3) / 4 <= FR_LDS_GRADT_ROWS_MAX;
  return (op.M + 3) / 4 <= FR_LDS_ROWS_MAX;
}

// Sparse-row candidates of one operator product (step 3 adds the fused
// gradient-transform plans).
void sparse_candidates(const GemmOp &op, int step, int D, std::vector<fr::GemmPlan> &cands) {
  if (!op.sp.colidx) return;
  if (staged_ok(op, false, D)) cands.push_back(fr::GemmPlan{0, 64, kPlanStaged});
  if (step == 3 && staged_ok(op, true, D))
    cands.push_back(fr::GemmPlan{0, 64, kPlanStaged | kPlanFusedGradT});
  // few rows per workgroup keep many workgroups on one column tile at once
  // (its B rows shared in L2); more rows amortise the operator loads
  for (int f : {0, kPlanFields})
    for (int rpg : {1, 2, 4, 8, 16, 32, 64}) cands.push_back(fr::GemmPlan{0, rpg, f});
  if (step == 3)
    for (int f : {0, kPlanFields, kPlanFields | kPlanFusedFlux}) {
      if (f && op.sp.width > FR_SPOP_GRADT_FIELDS_WMAX) continue;
      for (int rpg : {1, 2, 4, 8, 16}) cands.push_back(fr::GemmPlan{0, rpg, kPlanFusedGradT | f});
    }
}

struct BlockRT {
  int ref = 0;
  int etype = 0, order = 0;
  int64_t nelem = 0, ld = 0;
  int Nu = 0, Nf = 0;
  int64_t uoff = 0, ufoff = 0, qfoff = 0, ftoff = 0, part_off = 0;
  int64_t refoff = 0;  // reference states of the deviation form ([NV][ld])
  double *d_smat = nullptr, *d_rcpdjac = nullptr, *d_wdjac = nullptr;
  int32_t *d_prob = nullptr;
  GemmOp m0, m5, s3, s8;
  // transposed operators of the adjoint: M3^T, (M1 - M3 M2)^T, M0^T, M6^T,
  // [(M4 - M6 M0)^T | M0^T]
  GemmOp t_m3, t_m1, t_m0, t_m6, t_fin;
  std::vector<double> xu, wdjac_host;
};

// One launch of an operator product over several element blocks (steps 1,
// 5 and 8 of a mixed or batched mesh): the blocks whose plans share a
// kernel family, and a device table of their slots.
struct MultiLaunch {
  bool on = false;
  int width = 0, fields = 1;    // sparse-row family (precomputed gathers)
  int MBW = 0, NC = 0;          // matrix-core family
  std::vector<int> blocks;
  fr::LaunchSlot *d_slots = nullptr;
  int nslots = 0;
  int64_t nwg = 0;
  std::vector<void *> owned;    // slot table, padded operator copies, packed operators
};

// The transformed flux (step 6) over every block in one launch.
struct PointMulti {
  bool on = false;
  fr::PointSlot *d_slots = nullptr;
  int nslots = 0;
  int64_t nwg = 0;
};

}  // namespace

struct fr_ctx {
  fr_config cfg{};
  int D = 0, NV = 0;
  bool ns = false;
  bool no_fuse = false;  // run step 4 on its own even where step 3 would fuse it
  double *d_tune_dt = nullptr;  // zero step sizes (one per problem) for timing the RK epilogue
  int prec = 0;
  size_t tsize = 8;  // element size of the scratch arrays
  std::string err = "no error";
  std::vector<fr::RefOps> refs;
  std::vector<BlockRT> blocks;
  int64_t total_len = 0, uf_len = 0, qf_len = 0, ft_len = 0, nelem_total = 0;
  void *d_uf = nullptr, *d_qf = nullptr, *d_ft = nullptr;
  void *d_fto = nullptr;  // F~ (Navier-Stokes; Euler writes F~ over Q's storage)
  double *d_acc = nullptr, *d_stage = nullptr;
  // pairs
  int64_t npairs = 0;
  int32_t *d_lidx = nullptr, *d_ridx = nullptr, *d_lblk = nullptr, *d_rblk = nullptr;
  double *d_nrm = nullptr, *d_magL = nullptr, *d_magR = nullptr;
  // boundary flux points (Appendix C)
  int64_t nbpts = 0;
  int32_t *d_bidx = nullptr, *d_bblk = nullptr, *d_bcid = nullptr;
  double *d_bnrm = nullptr, *d_bmag = nullptr, *d_bcpar = nullptr;
  int64_t *d_blk_ufbase = nullptr, *d_blk_qfbase = nullptr, *d_blk_ld = nullptr,
          *d_blk_qstride = nullptr;
  // reductions
  double *d_part = nullptr, *d_part2 = nullptr;
  int64_t *d_pstart = nullptr, *d_plist = nullptr;
  // integral reductions: point ranges, slices per problem, list entries per slice
  int nchunk = 1, nslice = 1;
  int64_t slice_len = 64;
  int32_t *d_flag = nullptr;
  int nproblems = 1;
  // graphs of one and of kStepsPerGraph RK4 steps (same state and dt)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr, graph_k = nullptr;
  hipGraphExec_t graph_exec = nullptr, graph_k_exec = nullptr;
  const double *graph_u = nullptr, *graph_dt = nullptr;
  // adjoint scratch (allocated on first use, FP64 contexts only)
  // arrays the right-hand-side chain uses (default: the scratch above, with
  // D~ over U^f and F~ over Q as the paper aliases them; the stash path points
  // U^f, Q^f, Q into caller memory and the outputs into scratch)
  struct Bufs {
    void *uf, *qf, *ft, *df, *fto;
    double *stage_out;
    double *acc;  // RK register of the last-stage epilogue (null: d_acc)
  } cur{};
  bool adj_ready = false, adj_tuned = false;
  double *d_ufb = nullptr, *d_ftb = nullptr, *d_qfb = nullptr, *d_lt = nullptr;
  double *d_lc = nullptr, *d_w = nullptr, *d_k = nullptr;
  double *d_st[3] = {nullptr, nullptr, nullptr};
  // other steppers: forward Euler (one graph per step), DOPRI5 (slopes
  // k1..k7, the stage/new state y, per-problem error sums, DOF counts,
  // accept and rejection flags, one graph per attempt)
  hipGraph_t eu_graph = nullptr, eu_graph_k = nullptr;
  hipGraphExec_t eu_exec = nullptr, eu_exec_k = nullptr;
  const double *eu_u = nullptr, *eu_dt = nullptr;
  std::vector<double> ndof_host;
  bool dp_ready = false;
  double *d_dpk[7] = {};
  double *d_dpy = nullptr, *d_dp_ssq = nullptr, *d_dp_ndof = nullptr;
  int32_t *d_dp_acc = nullptr, *d_dp_rej = nullptr;
  hipGraph_t dp_graph = nullptr;
  hipGraphExec_t dp_exec = nullptr;
  struct DpKey {
    const double *u, *t, *dt, *tend;
    const int32_t *counts;
    double atol, rtol;
    bool operator==(const DpKey &o) const {
      return u == o.u && t == o.t && dt == o.dt && tend == o.tend && counts == o.counts &&
             atol == o.atol && rtol == o.rtol;
    }
  } dp_key{};
  // checkpoint segments of the adjoint (fr_rk_segment_adjoint): the replay
  // state and a few captured segment graphs, each keyed by its arguments
  double *d_seg_u = nullptr;
  struct SegGraph {
    const double *u0, *dt, *lam_end;
    double *lam0, *stash;
    int nsteps;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t used;
  };
  std::vector<SegGraph> seg_graphs;
  uint64_t seg_clock = 0;
  std::vector<void *> allocs;
  // Euler in reduced precision: the deviation form (each element's state
  // less its reference, the state at its first solution point, before any
  // rounding to FP32 or bf16)
  bool devform = false;
  void *d_udev = nullptr;        // u - u_ref (scratch element type, state layout)
  double *d_uref = nullptr;      // u_ref per block [NV][ld]
  int64_t *d_blk_refbase = nullptr;
  // multi-block launches: [step][family 0 sparse-row, 1 matrix cores]
  MultiLaunch multi[9][2];
  PointMulti tflux_multi;
};

namespace {

struct Fail {
  fr_status st;
  std::string msg;
};

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess)
    throw Fail{e == hipErrorOutOfMemory ? FR_ENOMEM : FR_EDEVICE,
               std::string(what) + ": " + hipGetErrorString(e)};
}

template <typename T>
T *dev_alloc(fr_ctx *c, size_t n) {
  void *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw Fail{FR_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
  c->allocs.push_back(p);
  hip_check(hipMemset(p, 0, n * sizeof(T)), "hipMemset");
  return (T *)p;
}

template <typename T>
T *dev_upload(fr_ctx *c, const T *h, size_t n, hipStream_t s) {
  T *d = dev_alloc<T>(c, n);
  if (n) hip_check(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s), "upload");
  hip_check(hipStreamSynchronize(s), "upload sync");
  return d;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// One row of a block's arrays (N_V ld values) is addressed with 32-bit byte
// offsets by the operator kernels, so it must span under 4 GiB.
bool block_too_large(const fr_block &B, int nvars) {
  return (int64_t)nvars * round_up(B.nelem, 16) >= ((int64_t)1 << 29);
}
const char *const kBlockTooLarge = "block too large: N_V * nelem must stay below 2^29; split it";

void *pack_upload(fr_ctx *c, const GemmOp &op, fr::GemmPlan p, hipStream_t s, bool track) {
  const bool bf = c->prec == FR_BF16X3;
  const int64_t n = bf ? fr::gemm_pack_size_bf16(op.M, op.K1, op.K2, p.MBW, p.WM)
                       : fr::gemm_pack_size(op.M, op.K1, op.K2, p.MBW, p.WM, 4);
  const size_t es = c->prec == FR_FP64 ? 8 : (bf ? 2 : 4);
  void *d = nullptr;
  hipError_t e = hipMalloc(&d, n * es);
  if (e != hipSuccess) throw Fail{FR_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
  if (track) c->allocs.push_back(d);
  if (c->prec == FR_FP64) {
    std::vector<double> pk(n);
    fr::gemm_pack_f64(op.A.data(), op.M, op.K1, op.K2, p.MBW, p.WM, pk.data());
    hip_check(hipMemcpyAsync(d, pk.data(), n * es, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "upload sync");
  } else if (bf) {
    std::vector<uint16_t> pk(n);
    fr::gemm_pack_bf16x3(op.A.data(), op.M, op.K1, op.K2, p.MBW, p.WM, pk.data());
    hip_check(hipMemcpyAsync(d, pk.data(), n * es, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "upload sync");
  } else {
    std::vector<float> pk(n);
    fr::gemm_pack_f32(op.A.data(), op.M, op.K1, op.K2, p.MBW, p.WM, pk.data());
    hip_check(hipMemcpyAsync(d, pk.data(), n * es, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "upload sync");
  }
  return d;
}

void make_op(fr_ctx *c, GemmOp &op, const std::vector<double> &A, int M, int K1, int K2,
             int64_t N, hipStream_t s, fr::GemmPlan *force = nullptr, int hint1 = 0,
             int hint2 = 0) {
  op.M = M; op.K1 = K1; op.K2 = K2;
  const int kstep = c->prec == FR_BF16X3 ? 32 : 4;
  op.KS1 = (K1 + kstep - 1) / kstep;
  op.KS2 = (K2 + kstep - 1) / kstep;
  op.A = A;
  // ELL copy (sparse-row kernel), FP64 and FP32 contexts
  {
    const int K = K1 + K2;
    std::vector<std::vector<int>> cols(M);
    size_t nnz = 0;
    int wmax = 1;
    for (int r = 0; r < M; ++r) {
      double mx = 0;
      for (int k = 0; k < K; ++k) mx = std::max(mx, std::fabs(A[(size_t)r * K + k]));
      for (int k = 0; k < K; ++k)
        if (std::fabs(A[(size_t)r * K + k]) > kSparseDrop * mx) cols[r].push_back(k);
      nnz += cols[r].size();
      wmax = std::max(wmax, (int)cols[r].size());
    }
    op.density = (double)nnz / ((double)M * K);
    const int W = fr::spop_width(wmax);
    if (c->prec != FR_BF16X3 && op.density < 0.5 && W > 0) {
      std::vector<int32_t> ci((size_t)M * W);
      std::vector<double> va((size_t)M * W, 0.0);
      for (int r = 0; r < M; ++r) {
        const int last = cols[r].empty() ? 0 : cols[r].back();
        for (int e = 0; e < W; ++e) {
          const bool real = e < (int)cols[r].size();
          ci[(size_t)r * W + e] = real ? cols[r][e] : last;
          va[(size_t)r * W + e] = real ? A[(size_t)r * K + cols[r][e]] : 0.0;
        }
      }
      op.sp.colidx = dev_upload(c, ci.data(), ci.size(), s);
      op.sp.vals = dev_upload(c, va.data(), va.size(), s);
      op.ell_cols = ci;
      op.ell_vals = va;
      op.sp.width = W;
      op.sp.rpg = 16;
      op.sp.fields = 1;
      // chunked copy for the LDS-staged kernel: each panel split into chunks
      // of at most kcmax rows of B (kStagedRows, or fewer where the device
      // allows a workgroup less LDS for 64 columns), aligned
      // where possible to the operator's blocks (hint1 rows of panel 1, such
      // as the points of one face; hint2 rows of panel 2, such as one
      // direction of the transformed flux), so that every operator row has
      // about the same number of entries in a chunk; columns within the chunk
      int maxshm = 32768;
      {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess)
          hipDeviceGetAttribute(&maxshm, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
      }
      // at most kStagedRows rows (64 KB of FP64 values) and what the device
      // allows a workgroup
      const int kcmax = std::max(
          16, std::min(fr::kStagedRows, maxshm / (64 * (c->prec == FR_FP64 ? 8 : 4))));
      std::vector<int> starts(1, 0);
      for (int pn = 0; pn < 2; ++pn) {
        const int rows = pn ? K2 : K1, hint = pn ? hint2 : hint1;
        if (rows <= 0) continue;
        int n = (rows + kcmax - 1) / kcmax;
        int size = 0;
        for (int m = n; hint > 0 && m <= rows && rows / m >= hint; ++m)
          if (rows % m == 0 && (rows / m) % hint == 0) { n = m; size = rows / m; break; }
        for (int i = 0; i < n; ++i)
          starts.push_back(starts.back() + (size ? size : rows / n + (i < rows % n)));
      }
      const int nchunk = (int)starts.size() - 1;
      int kc = 1;
      for (int ch = 0; ch < nchunk; ++ch) kc = std::max(kc, starts[ch + 1] - starts[ch]);
      std::vector<int32_t> cw(nchunk, 0);
      std::vector<int> chunk_of(K);
      for (int ch = 0; ch < nchunk; ++ch)
        for (int k = starts[ch]; k < starts[ch + 1]; ++k) chunk_of[k] = ch;
      for (int r = 0; r < M; ++r) {
        std::vector<int> cnt(nchunk, 0);
        for (int k : cols[r]) ++cnt[chunk_of[k]];
        for (int ch = 0; ch < nchunk; ++ch) cw[ch] = std::max(cw[ch], cnt[ch]);
      }
      const int WC = fr::spop_lds_width(*std::max_element(cw.begin(), cw.end()));
      if (WC > 0) {
        std::vector<int32_t> sci((size_t)nchunk * M * WC, 0);
        std::vector<double> sva((size_t)nchunk * M * WC, 0.0);
        for (int r = 0; r < M; ++r) {
          std::vector<int> fill(nchunk, 0);
          for (int k : cols[r]) {
            const int ch = chunk_of[k];
            const size_t at = ((size_t)ch * M + r) * WC + fill[ch]++;
            sci[at] = k - starts[ch];
            sva[at] = A[(size_t)r * K + k];
          }
        }
        op.st.colidx = dev_upload(c, sci.data(), sci.size(), s);
        op.st.vals = dev_upload(c, sva.data(), sva.size(), s);
        op.st.cstart = dev_upload(c, starts.data(), starts.size(), s);
        op.st.cwidth = dev_upload(c, cw.data(), cw.size(), s);
        op.st.width = WC;
        op.st.kc = kc;
        op.st.nchunk = nchunk;
      }
    }
  }
  fr::GemmPlan p = force ? *force : fr::gemm_plan(M, N, c->prec);
  if (p.MBW == 0 && !op.sp.colidx) p = fr::gemm_plan(M, N, c->prec);
  op.MBW = p.MBW; op.NC = p.NC; op.WM = p.WM;
  if (p.MBW == 0) {
    apply_sparse_plan(op, p, c->NV);
    op.d_A = nullptr;
  } else {
    op.d_A = pack_upload(c, op, p, s, true);
  }
}

// Step 3 with the gradient transform (step 4) fused into its epilogue: a
// sparse-row plan of the [M6|M4'] operator with WM = 1.
bool gradt_fused(const fr_ctx *c, const BlockRT &b) {
  return c->ns && !c->no_fuse && b.s3.MBW == 0 && (b.s3.WM & kPlanFusedGradT);
}

// Step 6 done in step 3's epilogue (needs F~ apart from Q: step 5 reads Q).
bool flux_fused(const fr_ctx *c, const BlockRT &b) {
  return gradt_fused(c, b) && (b.s3.WM & kPlanFusedAll) == kPlanFusedAll &&
         !(b.s3.WM & kPlanStaged) && c->cur.fto != c->cur.ft;
}

// Byte offsets of the B row of every ELL entry of `op`, for operands with
// row strides rs1 and rs2 bytes: k rs1 for a one-panel operator (from its
// panel, whatever its address); for two panels at B1 and B2, from the lower
// of the two.  Kept only if every entry's row, plus `span` bytes of columns,
// lies within 4 GiB of that base (one buffer resource covers both panels).
void build_row_offsets(fr_ctx *c, GemmOp &op, const void *B1, int64_t rs1, const void *B2,
                       int64_t rs2, int64_t span, hipStream_t s) {
  if (!op.sp.colidx || op.ell_cols.empty()) return;
  int64_t o1 = 0, o2 = 0;
  if (op.K2 > 0) {
    const int64_t d = (const char *)B2 - (const char *)B1;
    o1 = d < 0 ? -d : 0;
    o2 = d < 0 ? 0 : d;
    op.sp.roff_delta = d;
  }
  std::vector<uint32_t> off(op.ell_cols.size());
  for (size_t i = 0; i < off.size(); ++i) {
    const int k = op.ell_cols[i];
    const int64_t o = k < op.K1 ? o1 + (int64_t)k * rs1 : o2 + (int64_t)(k - op.K1) * rs2;
    if (o < 0 || o + span >= ((int64_t)1 << 32)) return;
    off[i] = (uint32_t)o;
  }
  op.sp.roff = dev_upload(c, off.data(), off.size(), s);
  op.roff_host = off;
  op.roff_rs1 = rs1;
  op.roff_rs2 = rs2;
}

// Launch an operator product with whichever kernel its plan names.  Sparse
// plans use the precomputed row offsets when they hold for these operands.
hipError_t launch_op(const GemmOp &op, int gprec, int epi, const fr::GemmArgs &g, int batch,
                     hipStream_t s) {
  if (op.MBW == 0 && (op.WM & kPlanStaged)) return fr::launch_spop_lds(gprec, epi, g, op.st, batch, s);
  if (op.MBW == 0) {
    if (op.sp.roff && g.ldb1 * (g.b1_f32 ? 4 : 8) == op.roff_rs1) {
      fr::GemmArgs go = g;
      if (op.K2 == 0) {
        go.roff = op.sp.roff; go.rbase = g.B1;
      } else if ((const char *)g.B2 - (const char *)g.B1 == op.sp.roff_delta &&
                 g.ldb2 * (g.b2_f32 ? 4 : 8) == op.roff_rs2) {
        go.roff = op.sp.roff; go.rbase = op.sp.roff_delta < 0 ? g.B2 : g.B1;
      }
      return fr::launch_spop(gprec, epi, go, op.sp, batch, s);
    }
    return fr::launch_spop(gprec, epi, g, op.sp, batch, s);
  }
  return fr::launch_gemm(gprec, epi, g, batch, s);
}

// concatenate two row-major matrices side by side: [A (M x K1) | B (M x K2)]
std::vector<double> hcat(const std::vector<double> &A, int K1, const std::vector<double> &B,
                         int K2, int M) {
  std::vector<double> out((size_t)M * (K1 + K2));
  for (int r = 0; r < M; ++r) {
    for (int k = 0; k < K1; ++k) out[(size_t)r * (K1 + K2) + k] = A[(size_t)r * K1 + k];
    for (int k = 0; k < K2; ++k) out[(size_t)r * (K1 + K2) + K1 + k] = B[(size_t)r * K2 + k];
  }
  return out;
}

fr_status fail(fr_ctx *c, fr_status st, const std::string &m) {
  if (c) c->err = m; else g_setup_error = m;
  return st;
}

void *elem(void *base, int64_t off, size_t ts) { return (char *)base + off * ts; }

fr::GemmArgs gemm_args(const GemmOp &op) {
  fr::GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.Apack = op.d_A; g.M = op.M; g.KS1 = op.KS1; g.KS2 = op.KS2; g.K1 = op.K1; g.K2 = op.K2;
  g.MBW = op.MBW; g.NC = op.NC; g.WM = op.WM;
  return g;
}

fr::PairArgs pair_args(fr_ctx *c) {
  fr::PairArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  const int NV = c->NV;
  pa.ndims = c->D; pa.nvars = NV; pa.npairs = c->npairs;
  pa.lidx = c->d_lidx; pa.ridx = c->d_ridx;
  pa.lblk = c->blocks.size() > 1 ? c->d_lblk : nullptr;
  pa.rblk = c->blocks.size() > 1 ? c->d_rblk : nullptr;
  pa.nrm = c->d_nrm; pa.magL = c->d_magL; pa.magR = c->d_magR;
  pa.uf = c->cur.uf; pa.uf_f32 = c->prec != FR_FP64; pa.cf = c->cur.qf; pa.qf = c->cur.qf;
  pa.dfout = c->cur.df != c->cur.uf ? c->cur.df : nullptr;
  pa.blk_ufbase = c->d_blk_ufbase; pa.blk_qfbase = c->d_blk_qfbase;
  pa.blk_ld = c->d_blk_ld; pa.blk_qstride = c->d_blk_qstride;
  pa.ld0 = c->blocks[0].ld;
  pa.qstride0 = (int64_t)c->blocks[0].Nf * NV * c->blocks[0].ld;
  pa.gamma = c->cfg.gamma; pa.mu = c->cfg.mu; pa.prandtl = c->cfg.prandtl;
  pa.beta = c->cfg.ldg_beta; pa.tau = c->cfg.ldg_tau;
  if (c->devform) {
    pa.uref = c->d_uref;
    pa.blk_refbase = c->d_blk_refbase;
  }
  return pa;
}

// Arguments of the boundary kernels: the boundary flux points as L sides.
fr::PairArgs bc_args(fr_ctx *c) {
  fr::PairArgs pa = pair_args(c);
  pa.npairs = c->nbpts;
  pa.lidx = c->d_bidx; pa.ridx = nullptr;
  pa.lblk = c->blocks.size() > 1 ? c->d_bblk : nullptr;
  pa.rblk = nullptr;
  pa.nrm = c->d_bnrm; pa.magL = c->d_bmag; pa.magR = nullptr;
  pa.bcid = c->d_bcid; pa.bcpar = c->d_bcpar;
  return pa;
}

fr::PointArgs point_args(fr_ctx *c, const BlockRT &b, const double *u) {
  fr::PointArgs p;
  std::memset(&p, 0, sizeof(p));
  p.ndims = c->D; p.nvars = c->NV; p.nupts = b.Nu; p.ld = b.ld; p.nelem = b.nelem;
  p.smat = b.d_smat; p.rcpdjac = b.d_rcpdjac; p.u = u + b.uoff;
  p.q = elem(c->cur.ft, b.ftoff, c->tsize); p.q_f32 = c->prec != FR_FP64;
  p.fout = c->cur.fto != c->cur.ft ? elem(c->cur.fto, b.ftoff, c->tsize) : nullptr;
  p.gamma = c->cfg.gamma; p.mu = c->cfg.mu; p.prandtl = c->cfg.prandtl;
  if (c->devform) {
    p.udev = elem(c->d_udev, b.uoff, c->tsize);
    p.uref = c->d_uref + b.refoff;
  }
  return p;
}

// ---------------------------------------------------------------------------
// Multi-block launches
// ---------------------------------------------------------------------------
GemmOp &step_op(BlockRT &b, int st) { return st == 1 ? b.m0 : st == 5 ? b.m5 : b.s8; }

template <typename T>
T *owned_upload(MultiLaunch &ml, const T *h, size_t n, hipStream_t s) {
  void *d = nullptr;
  hip_check(hipMalloc(&d, std::max<size_t>(1, n) * sizeof(T)), "hipMalloc");
  ml.owned.push_back(d);
  hip_check(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s), "upload");
  hip_check(hipStreamSynchronize(s), "upload sync");
  return (T *)d;
}

// Element offsets of block b's operands for step st (slot of a
// multi-block launch): step 1 reads the state and writes U^f; step 5 reads
// Q and writes Q^f (D batch slices); step 8 reads D~ and F~ and updates the
// state registers.
void slot_offsets(const fr_ctx *c, const BlockRT &b, int st, fr::LaunchSlot &sl) {
  const int64_t N = (int64_t)c->NV * b.ld;
  sl.ld = b.ld; sl.N = N; sl.nelem = b.nelem;
  sl.rcpdjac = b.d_rcpdjac; sl.prob = b.d_prob;
  if (st == 1) {
    sl.off_b1 = b.uoff; sl.off_c = b.ufoff;
  } else if (st == 5) {
    sl.off_b1 = b.ftoff; sl.off_c = b.qfoff;
    sl.sB1 = (int64_t)b.Nu * N; sl.sC = (int64_t)b.Nf * N;
  } else {
    sl.off_b1 = b.ufoff; sl.off_b2 = b.ftoff; sl.off_u = b.uoff;
  }
}

// Blocks of step st whose plan is in the family (0: sparse-row with
// precomputed gathers, 1: matrix cores, FP64 and FP32 contexts).
std::vector<int> family_blocks(fr_ctx *c, int st, int fam) {
  std::vector<int> out;
  for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
    GemmOp &op = step_op(c->blocks[bi], st);
    if (fam == 0 && op.MBW == 0 && !(op.WM & kPlanStaged) && op.sp.roff &&
        op.ell_vals.size() == op.roff_host.size())
      out.push_back((int)bi);
    if (fam == 1 && op.MBW > 0 && c->prec != FR_BF16X3) out.push_back((int)bi);
  }
  return out;
}

void free_multi(MultiLaunch &ml) {
  for (void *p : ml.owned) hipFree(p);
  ml = MultiLaunch{};
}

// One sparse-row launch over the family's blocks with `fields` fields per
// thread: every block's ELL padded to the widest (padding: value 0 on the
// row's last real entry), its own rows per workgroup row.
bool build_multi_sparse(fr_ctx *c, int st, int fields, hipStream_t s) {
  MultiLaunch &ml = c->multi[st][0];
  free_multi(ml);
  const std::vector<int> bl = family_blocks(c, st, 0);
  if (bl.size() < 2) return false;
  int W = 0;
  for (int bi : bl) W = std::max(W, step_op(c->blocks[bi], st).sp.width);
  std::vector<fr::LaunchSlot> host;
  int64_t wg = 0;
  for (int bi : bl) {
    BlockRT &b = c->blocks[bi];
    GemmOp &op = step_op(b, st);
    const int w0 = op.sp.width, M = op.M;
    const double *dv = op.sp.vals;
    const uint32_t *dr = op.sp.roff;
    if (w0 != W) {
      std::vector<double> v((size_t)M * W, 0.0);
      std::vector<uint32_t> r((size_t)M * W);
      for (int row = 0; row < M; ++row)
        for (int e = 0; e < W; ++e) {
          const size_t src = (size_t)row * w0 + std::min(e, w0 - 1);
          v[(size_t)row * W + e] = e < w0 ? op.ell_vals[src] : 0.0;
          r[(size_t)row * W + e] = op.roff_host[src];
        }
      dv = owned_upload(ml, v.data(), v.size(), s);
      dr = owned_upload(ml, r.data(), r.size(), s);
    }
    fr::LaunchSlot sl{};
    slot_offsets(c, b, st, sl);
    sl.wg_begin = wg;
    sl.vals = dv; sl.roff = dr;
    sl.rbase_b2 = op.K2 > 0 && op.sp.roff_delta < 0;
    sl.M = M; sl.K1 = op.K1; sl.K2 = op.K2;
    sl.rpg = op.sp.rpg;
    sl.ngroups = (M + sl.rpg - 1) / sl.rpg;
    wg += fr::spop_workgroups(fields == 1 ? sl.N : b.ld, M, sl.rpg);
    host.push_back(sl);
  }
  ml.d_slots = owned_upload(ml, host.data(), host.size(), s);
  ml.nslots = (int)host.size(); ml.nwg = wg; ml.blocks = bl;
  ml.width = W; ml.fields = fields; ml.on = true;
  return true;
}

// One matrix-core launch over the family's blocks: the largest tuned row
// blocks per wavefront, NC column strips, each block's operator packed for
// its own row split.
bool build_multi_mfma(fr_ctx *c, int st, int NC, hipStream_t s) {
  MultiLaunch &ml = c->multi[st][1];
  free_multi(ml);
  const std::vector<int> bl = family_blocks(c, st, 1);
  if (bl.size() < 2) return false;
  int MBW = 0;
  for (int bi : bl) MBW = std::max(MBW, step_op(c->blocks[bi], st).MBW);
  if (!fr::gemm_plan_valid(MBW, NC)) return false;
  std::vector<fr::LaunchSlot> host;
  int64_t wg = 0;
  for (int bi : bl) {
    BlockRT &b = c->blocks[bi];
    GemmOp &op = step_op(b, st);
    const int WM = (op.M + 16 * MBW - 1) / (16 * MBW);
    void *A = pack_upload(c, op, fr::GemmPlan{MBW, NC, WM}, s, false);
    ml.owned.push_back(A);
    fr::LaunchSlot sl{};
    slot_offsets(c, b, st, sl);
    sl.wg_begin = wg;
    sl.Apack = A;
    sl.M = op.M; sl.K1 = op.K1; sl.K2 = op.K2; sl.KS1 = op.KS1; sl.KS2 = op.KS2; sl.WM = WM;
    wg += fr::gemm_workgroups(sl.N, NC, WM);
    host.push_back(sl);
  }
  ml.d_slots = owned_upload(ml, host.data(), host.size(), s);
  ml.nslots = (int)host.size(); ml.nwg = wg; ml.blocks = bl;
  ml.MBW = MBW; ml.NC = NC; ml.on = true;
  return true;
}

// The transformed flux over every block in one launch (blocks whose flux is
// not fused into step 3).
bool build_tflux_multi(fr_ctx *c, hipStream_t s) {
  PointMulti &pm = c->tflux_multi;
  pm.on = false;
  if (c->blocks.size() < 2) return false;
  for (auto &b : c->blocks)
    if (flux_fused(c, b)) return false;
  std::vector<fr::PointSlot> host;
  int64_t wg = 0;
  for (auto &b : c->blocks) {
    fr::PointSlot sl{};
    sl.wg_begin = wg;
    sl.off_u = b.uoff; sl.off_q = b.ftoff; sl.off_ref = b.refoff;
    sl.nupts = b.Nu; sl.ld = b.ld; sl.nelem = b.nelem;
    sl.smat = b.d_smat; sl.rcpdjac = b.d_rcpdjac;
    wg += fr::point_workgroups(b.Nu, b.ld);
    host.push_back(sl);
  }
  if (!pm.d_slots) pm.d_slots = dev_upload(c, host.data(), host.size(), s);
  pm.nslots = (int)host.size(); pm.nwg = wg; pm.on = true;
  return true;
}

// The one-launch transformed flux needs every block's flux unfused (a plan
// forced later may fuse it into step 3).
bool tflux_multi_valid(const fr_ctx *c) {
  for (auto &b : c->blocks)
    if (flux_fused(c, b)) return false;
  return true;
}

// Whether a multi-block launch of step st applies to the arrays in use: the
// two-panel product's precomputed offsets assume the context's own D~ and F~.
bool multi_usable(const fr_ctx *c, int st) {
  if (st != 8) return true;
  return c->cur.df == c->d_uf && c->cur.fto == (c->ns ? c->d_fto : c->d_ft);
}

// Issue the multi-block launches of step st; marks the blocks they cover.
void run_multi(fr_ctx *c, int st, const double *u, double *dudt, int epi, const fr::RkCoef *rk,
               const double *dt, hipStream_t s, std::vector<char> &done) {
  if (!multi_usable(c, st)) return;
  const int f32 = c->prec != FR_FP64;
  const int gprec = c->prec == FR_FP64 ? fr::PREC_F64 : fr::PREC_F32;
  // the chain's epilogue (-1/J or the RK4 update) belongs to step 8; steps
  // 1 and 5 store their products, as their launches per block do
  const int sepi = st == 8 ? epi : fr::EPI_STORE;
  for (int fam = 0; fam < 2; ++fam) {
    MultiLaunch &ml = c->multi[st][fam];
    if (!ml.on) continue;
    fr::GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.slots = ml.d_slots; g.nslots = ml.nslots; g.nwg = ml.nwg;
    int batch = 1;
    if (st == 1) {
      g.B1 = c->devform ? (const void *)c->d_udev : (const void *)u;
      g.b1_f32 = g.b2_f32 = c->devform ? 1 : 0;
      g.C = c->cur.uf; g.c_f32 = f32;
    } else if (st == 5) {
      g.B1 = c->cur.ft; g.b1_f32 = f32; g.b2_f32 = f32;
      g.C = c->cur.qf; g.c_f32 = f32;
      batch = c->D;
    } else {
      g.B1 = c->cur.df; g.b1_f32 = f32;
      g.B2 = c->cur.fto; g.b2_f32 = f32;
      g.out = dudt;
      g.K2 = 1;  // two panels
      if (epi == fr::EPI_RK) {
        g.acc = c->cur.acc ? c->cur.acc : c->d_acc;
        g.stage = c->cur.stage_out;
        g.dt = dt; g.rk = *rk;
      }
    }
    if (fam == 0) {
      hip_check(fr::launch_spop_multi(gprec, sepi, g, ml.width, ml.fields, batch, s),
                "multi-block sparse-row product");
    } else {
      // g.N is per slot; any positive value passes the launcher's empty check
      g.MBW = ml.MBW; g.NC = ml.NC; g.N = 1;
      hip_check(fr::launch_gemm(gprec, sepi, g, batch, s), "multi-block matrix-core product");
    }
    for (int bi : ml.blocks) done[bi] = 1;
  }
}

// Steps of the right-hand side (every block):
//   1  U^f = M0 U                         (S1, GEMM)
//   2  C^f = common solution               (S2, pairs; Navier-Stokes)
//   3  Q~ = M6 C^f + (M4 - M6 M0) U        (S3, GEMM; Navier-Stokes)
//   4  Q = J^-T Q~ in place                (S4; Navier-Stokes)
//   5  Q^f = blockdiag(M0) Q               (S5, GEMM; Navier-Stokes)
//   6  F~ = J J^-1 f(U, Q)                 (S6; over Q's storage)
//   7  D~ = common normal flux, over U^f   (S7, pairs)
//   8  R = -J^-1 (M3 D~ + (M1 - M3 M2) F~) (S8 + S9, GEMM; + S10 with EPI_RK)
void run_step(fr_ctx *c, int st, const double *u, double *dudt, int epi, const fr::RkCoef *rk,
              const double *dt, hipStream_t s) {
  const int D = c->D, NV = c->NV;
  const size_t ts = c->tsize;
  const int f32 = c->prec != FR_FP64;
  const int gprec = c->prec == FR_FP64 ? fr::PREC_F64
                    : (c->prec == FR_FP32 ? fr::PREC_F32 : fr::PREC_BF16X3);
  if (!c->ns && st >= 2 && st <= 5) return;
  if (st == 2) {
    hip_check(fr::launch_con_u(pair_args(c), s), "con_u");
    if (c->nbpts) hip_check(fr::launch_bc_con_u(bc_args(c), s), "boundary con_u");
    return;
  }
  if (st == 7) {
    hip_check(fr::launch_comm_flux(pair_args(c), c->ns, s), "comm_flux");
    if (c->nbpts) hip_check(fr::launch_bc_comm_flux(bc_args(c), c->ns, s), "boundary comm_flux");
    return;
  }
  // one launch per kernel family over several blocks where set up
  std::vector<char> done(c->blocks.size(), 0);
  if (st == 1 || st == 5 || st == 8) run_multi(c, st, u, dudt, epi, rk, dt, s, done);
  if (st == 6 && c->tflux_multi.on && tflux_multi_valid(c)) {
    fr::PointArgs a = point_args(c, c->blocks[0], u);
    a.u = u;
    a.q = c->cur.ft;
    a.fout = c->cur.fto != c->cur.ft ? c->cur.fto : nullptr;
    if (c->devform) {
      a.udev = c->d_udev;
      a.uref = c->d_uref;
    }
    a.slots = c->tflux_multi.d_slots; a.nslots = c->tflux_multi.nslots; a.nwg = c->tflux_multi.nwg;
    hip_check(fr::launch_tflux(a, c->ns, s), "multi-block tflux");
    return;
  }
  for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
    if (done[bi]) continue;
    BlockRT &b = c->blocks[bi];
    const int64_t N = NV * b.ld;
    if (st == 1) {
      fr::GemmArgs g = gemm_args(b.m0);
      g.ld = b.ld;
      if (c->devform) {
        // one panel: B2 is never read, typed as B1 so that both panels share
        // an element size (precomputed-gather kernels)
        g.B1 = elem(c->d_udev, b.uoff, ts); g.ldb1 = N; g.b1_f32 = 1; g.b2_f32 = 1;
      } else {
        g.B1 = u + b.uoff; g.ldb1 = N; g.b1_f32 = 0;
      }
      g.C = elem(c->cur.uf, b.ufoff, ts); g.ldc = N; g.c_f32 = f32;
      g.N = N;
      hip_check(launch_op(b.m0, gprec, fr::EPI_STORE, g, 1, s), "gemm M0");
    } else if (st == 0) {
      // deviation form (Navier-Stokes): the state's deviation and reference
      hip_check(fr::launch_devstate(point_args(c, b, u), s), "deviation");
    } else if (st == 3) {
      fr::GemmArgs g = gemm_args(b.s3);
      g.ld = b.ld;
      g.B1 = elem(c->cur.qf, b.qfoff, ts); g.ldb1 = N; g.b1_f32 = f32;
      // the gradient of the state from its deviation in the deviation form
      // (the reference is constant in the element)
      if (c->devform) {
        g.B2 = elem(c->d_udev, b.uoff, ts); g.ldb2 = N; g.b2_f32 = 1;
      } else {
        g.B2 = u + b.uoff; g.ldb2 = N; g.b2_f32 = 0;
      }
      g.uprim = u + b.uoff; g.devflux = c->devform ? 1 : 0;
      g.C = elem(c->cur.ft, b.ftoff, ts); g.ldc = N; g.c_f32 = f32;
      g.N = N;
      if (gradt_fused(c, b)) {
        g.rcpdjac = b.d_rcpdjac; g.ld = b.ld; g.nelem = b.nelem;
        g.smat = b.d_smat; g.D = D; g.Nu = b.Nu;
        if (flux_fused(c, b)) {
          g.fout = elem(c->cur.fto, b.ftoff, ts);
          g.gamma = c->cfg.gamma; g.mu = c->cfg.mu; g.prandtl = c->cfg.prandtl;
          hip_check(launch_op(b.s3, gprec, fr::EPI_GRADTF, g, 1, s), "gemm M6|M4' + J^-T + flux");
        } else {
          hip_check(launch_op(b.s3, gprec, fr::EPI_GRADT, g, 1, s), "gemm M6|M4' + J^-T");
        }
      } else {
        hip_check(launch_op(b.s3, gprec, fr::EPI_STORE, g, 1, s), "gemm M6|M4'");
      }
    } else if (st == 4) {
      if (!gradt_fused(c, b))
        hip_check(fr::launch_gradcoru(point_args(c, b, u), s), "gradcoru");
    } else if (st == 5) {
      fr::GemmArgs g = gemm_args(b.m5);
      g.ld = b.ld;
      g.B1 = elem(c->cur.ft, b.ftoff, ts); g.ldb1 = N; g.b1_f32 = f32; g.b2_f32 = f32;
      g.C = elem(c->cur.qf, b.qfoff, ts); g.ldc = N; g.c_f32 = f32;
      g.N = N;
      g.sB1 = (int64_t)b.Nu * N;
      g.sC = (int64_t)b.Nf * N;
      hip_check(launch_op(b.m5, gprec, fr::EPI_STORE, g, D, s), "gemm M5");
    } else if (st == 6) {
      if (!flux_fused(c, b))
        hip_check(fr::launch_tflux(point_args(c, b, u), c->ns, s), "tflux");
    } else if (st == 8) {
      fr::GemmArgs g = gemm_args(b.s8);
      g.B1 = elem(c->cur.df, b.ufoff, ts); g.ldb1 = N; g.b1_f32 = f32;
      g.B2 = elem(c->cur.fto, b.ftoff, ts); g.ldb2 = N; g.b2_f32 = f32;
      g.ldc = N; g.N = N;
      g.rcpdjac = b.d_rcpdjac; g.ld = b.ld; g.nelem = b.nelem;
      g.out = dudt + b.uoff;
      if (epi == fr::EPI_RK) {
        g.acc = (c->cur.acc ? c->cur.acc : c->d_acc) + b.uoff;
        g.stage = c->cur.stage_out ? c->cur.stage_out + b.uoff : nullptr;
        g.dt = dt; g.prob = b.d_prob; g.rk = *rk;
      }
      hip_check(launch_op(b.s8, gprec, epi, g, 1, s), "gemm M3|M1'");
    }
  }
}

// The right-hand-side chain, steps 1..min(stop, 8).  epi: EPI_NEGDIV writes
// dudt; EPI_RK applies the RK stage update `rk` with registers (dudt = u,
// acc, stage).
// Order of the steps: the deviation form computes the transformed flux
// first, since it also writes the deviations step 1 interpolates.
const std::vector<int> &chain_order(const fr_ctx *c) {
  // deviation form: Euler writes the state's deviation with the flux (step
  // 6 first); Navier-Stokes needs it before step 1, from a pass of its own
  // (step 0), and takes the flux after the gradient as usual
  static const std::vector<int> plain{1, 2, 3, 4, 5, 6, 7, 8}, dev{6, 1, 7, 8},
      dev_ns{0, 1, 2, 3, 4, 5, 6, 7, 8};
  return !c->devform ? plain : c->ns ? dev_ns : dev;
}

// The right-hand-side chain in its order, up to and including step `stop`
// (stop < 0: nothing; 0 is the deviation pass of Navier-Stokes in the
// deviation form).
void rhs_chain(fr_ctx *c, const double *u, double *dudt, int epi, const fr::RkCoef *rk,
               const double *dt, hipStream_t s, int stop = 8) {
  if (stop < 0) return;
  for (int st : chain_order(c)) {
    run_step(c, st, u, dudt, epi, rk, dt, s);
    if (st == stop) break;
  }
}

// The step just before `step` in the chain's order (the chain up to it
// makes step's inputs); -1 if none.
int step_before(const fr_ctx *c, int step) {
  const std::vector<int> &o = chain_order(c);
  for (size_t i = 0; i < o.size(); ++i)
    if (o[i] == step) return i ? o[i - 1] : -1;
  return -1;
}

// Time every instantiated plan of each operator product on this mesh (the
// real scratch arrays as operands, HIP events on the set-up stream) and keep
// the fastest.  Results are memoised per shape for the process.
struct TuneKey {
  int prec, M, K1, K2, batch, epi, step;
  int64_t N;
  bool operator<(const TuneKey &o) const {
    return std::tie(prec, M, K1, K2, batch, epi, step, N) <
           std::tie(o.prec, o.M, o.K1, o.K2, o.batch, o.epi, o.step, o.N);
  }
};
std::map<TuneKey, fr::GemmPlan> g_tuned;

void tune_op(fr_ctx *c, GemmOp &op, int step, BlockRT &b, hipStream_t s) {
  const int batch = step == 5 ? c->D : 1;
  // step 8 is timed with the RK4 stage update the captured step graph uses
  // (a middle stage: reads u and acc, writes acc and the next stage); the
  // values are meaningless (dt = 0 from d_tune_dt), the traffic is the same
  const int epi = step == 8 ? fr::EPI_RK : fr::EPI_STORE;
  fr::RkCoef rk;
  rk.a_next = 0.5; rk.b = 1.0 / 3; rk.first = 0; rk.last = 0;
  const fr::RkCoef *rkp = step == 8 ? &rk : nullptr;
  const double *dtp = step == 8 ? c->d_tune_dt : nullptr;
  const int64_t N = (int64_t)c->NV * b.ld;
  TuneKey key{c->prec, op.M, op.K1, op.K2, batch, epi, step, N};
  fr::GemmPlan best{op.MBW, op.NC, op.WM};
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    best = it->second;
  } else {
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    float best_ms = 1e30f;
    std::vector<fr::GemmPlan> cands = fr::gemm_candidates(op.M, N, c->prec);
    // step 3: also the plans with the gradient transform (and the flux)
    // fused; every candidate is timed together with steps 4 and 6 (no-ops
    // when fused)
    sparse_candidates(op, step, c->D, cands);
    for (const fr::GemmPlan &p : cands) {
      void *d = p.MBW ? pack_upload(c, op, p, s, false) : nullptr;
      GemmOp trial = op;
      trial.d_A = d; trial.MBW = p.MBW; trial.NC = p.NC; trial.WM = p.WM;
      if (p.MBW == 0) apply_sparse_plan(trial, p, c->NV);
      std::swap(*(step == 1 ? &b.m0 : step == 3 ? &b.s3 : step == 5 ? &b.m5 : &b.s8), trial);
      float ms = 0;
      try {
        for (int w = 0; w < 2; ++w) {
          run_step(c, step, c->d_stage, c->d_acc, epi, rkp, dtp, s);
          if (step == 3) {
            run_step(c, 4, c->d_stage, c->d_acc, epi, nullptr, nullptr, s);
            run_step(c, 6, c->d_stage, c->d_acc, epi, nullptr, nullptr, s);
          }
        }
        hip_check(hipEventRecord(e0, s), "record");
        for (int w = 0; w < 5; ++w) {
          run_step(c, step, c->d_stage, c->d_acc, epi, rkp, dtp, s);
          if (step == 3) {
            run_step(c, 4, c->d_stage, c->d_acc, epi, nullptr, nullptr, s);
            run_step(c, 6, c->d_stage, c->d_acc, epi, nullptr, nullptr, s);
          }
        }
        hip_check(hipEventRecord(e1, s), "record");
        hip_check(hipEventSynchronize(e1), "sync");
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
      } catch (...) {
        std::swap(*(step == 1 ? &b.m0 : step == 3 ? &b.s3 : step == 5 ? &b.m5 : &b.s8), trial);
        hipFree(d);
        throw;
      }
      std::swap(*(step == 1 ? &b.m0 : step == 3 ? &b.s3 : step == 5 ? &b.m5 : &b.s8), trial);
      hipFree(d);
      if (ms < best_ms) { best_ms = ms; best = p; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    g_tuned[key] = best;
  }
  if (best.MBW != op.MBW || best.NC != op.NC || best.WM != op.WM) {
    op.d_A = best.MBW ? pack_upload(c, op, best, s, true) : nullptr;
    op.MBW = best.MBW; op.NC = best.NC; op.WM = best.WM;
    if (best.MBW == 0) apply_sparse_plan(op, best, c->NV);
  }
}

// One launch per kernel family over the blocks of a multi-block mesh, kept
// by the set-up where it is not slower than a launch per block.
constexpr bool kMultiBlockLaunches = true;

// Mean time of step st over 5 launches (after 2), with the RK epilogue the
// step graph uses for step 8 (dt = 0: values meaningless, traffic the same).
float time_step_ms(fr_ctx *c, int st, hipStream_t s) {
  const int epi = st == 8 ? fr::EPI_RK : fr::EPI_STORE;
  fr::RkCoef rk;
  rk.a_next = 0.5; rk.b = 1.0 / 3; rk.first = 0; rk.last = 0;
  const fr::RkCoef *rkp = st == 8 ? &rk : nullptr;
  const double *dtp = st == 8 ? c->d_tune_dt : nullptr;
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  float ms = 0;
  try {
    for (int w = 0; w < 2; ++w) run_step(c, st, c->d_stage, c->d_acc, epi, rkp, dtp, s);
    hip_check(hipEventRecord(e0, s), "record");
    for (int w = 0; w < 5; ++w) run_step(c, st, c->d_stage, c->d_acc, epi, rkp, dtp, s);
    hip_check(hipEventRecord(e1, s), "record");
    hip_check(hipEventSynchronize(e1), "sync");
    hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
  } catch (...) {
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    throw;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms / 5;
}

// Steps 1, 5, 8 and 6 of a multi-block mesh: one launch per kernel family
// over its blocks (each block keeping its tuned rows per workgroup, or its
// row split), kept where it is not slower than a launch per block; for the
// sparse-row family one or all fields per thread, for the matrix cores 1,
// 2 or 4 column strips per wavefront.
void tune_multi(fr_ctx *c, hipStream_t s) {
  if (c->blocks.size() < 2 || c->prec == FR_BF16X3) return;
  for (int st : {1, 5, 8}) {
    if (st == 5 && !c->ns) continue;
    free_multi(c->multi[st][0]);
    free_multi(c->multi[st][1]);
    float best = time_step_ms(c, st, s);
    int bestF = 0;
    for (int F : {1, c->NV})
      if (build_multi_sparse(c, st, F, s)) {
        const float t = time_step_ms(c, st, s);
        if (t <= best) { best = t; bestF = F; }
      }
    if (bestF) build_multi_sparse(c, st, bestF, s);
    else free_multi(c->multi[st][0]);
    int bestNC = 0;
    for (int NC : {1, 2, 4})
      if (build_multi_mfma(c, st, NC, s)) {
        const float t = time_step_ms(c, st, s);
        if (t <= best) { best = t; bestNC = NC; }
      }
    if (bestNC) build_multi_mfma(c, st, bestNC, s);
    else free_multi(c->multi[st][1]);
  }
  c->tflux_multi.on = false;
  const float t_sep = time_step_ms(c, 6, s);
  if (build_tflux_multi(c, s) && time_step_ms(c, 6, s) > t_sep) c->tflux_multi.on = false;
}

void autotune(fr_ctx *c, hipStream_t s) {
  for (auto &b : c->blocks) {
    tune_op(c, b.m0, 1, b, s);
    tune_op(c, b.s8, 8, b, s);
    if (c->ns) {
      tune_op(c, b.s3, 3, b, s);
      tune_op(c, b.m5, 5, b, s);
    }
  }
  // one launch per kernel family over several blocks
  if (kMultiBlockLaunches) tune_multi(c, s);
  hip_check(hipStreamSynchronize(s), "tune sync");
}

std::vector<double> transpose(const std::vector<double> &A, int rows, int cols) {
  std::vector<double> T((size_t)rows * cols);
  for (int r = 0; r < rows; ++r)
    for (int c2 = 0; c2 < cols; ++c2) T[(size_t)c2 * rows + r] = A[(size_t)r * cols + c2];
  return T;
}

void ensure_adjoint(fr_ctx *c, hipStream_t s) {
  if (c->nbpts) throw Fail{FR_EUNSUPPORTED, "the adjoint does not cover boundary conditions"};
  if (c->adj_ready) return;
  if (c->prec != FR_FP64) throw Fail{FR_EUNSUPPORTED, "the adjoint is available for FP64 contexts"};
  const int D = c->D, NV = c->NV;
  c->d_ufb = dev_alloc<double>(c, c->uf_len);
  c->d_ftb = dev_alloc<double>(c, c->ft_len);
  if (c->ns) c->d_qfb = dev_alloc<double>(c, c->qf_len);
  for (double **p : {&c->d_lt, &c->d_lc, &c->d_w, &c->d_k, &c->d_st[0], &c->d_st[1], &c->d_st[2]})
    *p = dev_alloc<double>(c, c->total_len);
  for (auto &b : c->blocks) {
    const fr::RefOps &R = c->refs[b.ref];
    const int Nu = R.nupts, Nf = R.nfpts;
    const int64_t N = (int64_t)NV * b.ld;
    make_op(c, b.t_m3, transpose(R.M3, Nu, Nf), Nf, Nu, 0, N, s);
    make_op(c, b.t_m1, transpose(R.M1p, Nu, D * Nu), D * Nu, Nu, 0, N, s);
    make_op(c, b.t_m0, transpose(R.M0, Nf, Nu), Nu, Nf, 0, c->ns ? D * N : N, s);
    if (c->ns) {
      make_op(c, b.t_m6, transpose(R.M6, D * Nu, Nf), Nf, D * Nu, 0, N, s);
      make_op(c, b.t_fin, hcat(transpose(R.M4p, D * Nu, Nu), D * Nu, transpose(R.M0, Nf, Nu), Nf, Nu),
              Nu, D * Nu, Nf, N, s);
    }
  }
  c->adj_ready = true;
  c->adj_tuned = !c->cfg.autotune;
}

fr::AdjPairArgs adj_pair_args(fr_ctx *c) {
  fr::AdjPairArgs a;
  std::memset(&a, 0, sizeof(a));
  const int NV = c->NV;
  a.ndims = c->D; a.nvars = NV; a.npairs = c->npairs;
  a.lidx = c->d_lidx; a.ridx = c->d_ridx;
  a.lblk = c->blocks.size() > 1 ? c->d_lblk : nullptr;
  a.rblk = c->blocks.size() > 1 ? c->d_rblk : nullptr;
  a.nrm = c->d_nrm; a.magL = c->d_magL; a.magR = c->d_magR;
  a.uf = (const double *)c->d_uf; a.qf = (const double *)c->d_qf;
  a.ufb = c->d_ufb; a.qfb = c->d_qfb;
  a.blk_ufbase = c->d_blk_ufbase; a.blk_qfbase = c->d_blk_qfbase;
  a.blk_ld = c->d_blk_ld; a.blk_qstride = c->d_blk_qstride;
  a.ld0 = c->blocks[0].ld;
  a.qstride0 = (int64_t)c->blocks[0].Nf * NV * c->blocks[0].ld;
  a.gamma = c->cfg.gamma; a.mu = c->cfg.mu; a.prandtl = c->cfg.prandtl;
  a.beta = c->cfg.ldg_beta; a.tau = c->cfg.ldg_tau;
  return a;
}

void adj_gemm(fr_ctx *c, const GemmOp &op, const double *B1, const double *B2, double *C,
              int64_t N, int epi, int batch, int64_t sB1, int64_t sC, hipStream_t s) {
  fr::GemmArgs g = gemm_args(op);
  g.B1 = B1; g.ldb1 = N; g.B2 = B2; g.ldb2 = N;
  g.C = C; g.ldc = N; g.N = N; g.sB1 = sB1; g.sC = sC;
  g.ld = N / c->NV;  // columns are (field, element) with N = N_V ld
  hip_check(launch_op(op, fr::PREC_F64, epi, g, batch, s), "adjoint gemm");
}

// Autotune one transposed operator of the adjoint with its real operands.
bool tfvjp_fused(const BlockRT &b) {
  return b.t_m1.MBW == 0 && (b.t_m1.WM & (kPlanFields | kPlanFusedFluxVjp)) ==
                               (kPlanFields | kPlanFusedFluxVjp);
}

// (M1 - M3 M2)^T lt with the reverse of the transformed flux in the
// epilogue: the state cotangent into ulam, Qb (Navier-Stokes) over F~b.
void adj_m1t_fused(fr_ctx *c, const BlockRT &b, const GemmOp &op, const double *u,
                   const double *qprim, double *ulam, hipStream_t s) {
  const int64_t N = (int64_t)c->NV * b.ld;
  fr::GemmArgs g = gemm_args(op);
  g.B1 = c->d_lt + b.uoff; g.ldb1 = N; g.B2 = nullptr; g.ldb2 = N;
  g.C = c->d_ftb + b.ftoff; g.ldc = N; g.N = N;
  g.ld = b.ld; g.nelem = b.nelem; g.rcpdjac = b.d_rcpdjac;
  g.smat = b.d_smat; g.D = c->D; g.Nu = b.Nu;
  g.uprim = u + b.uoff; g.qprim = c->ns && qprim ? qprim + b.ftoff : nullptr;
  g.out = ulam + b.uoff;
  g.gamma = c->cfg.gamma; g.mu = c->cfg.mu; g.prandtl = c->cfg.prandtl;
  hip_check(launch_op(op, fr::PREC_F64, fr::EPI_TFVJP, g, 1, s), "adjoint gemm + flux VJP");
}

void tune_adj(fr_ctx *c, GemmOp &op, const double *B1, const double *B2, double *C, int64_t N,
              int epi, int batch, int64_t sB1, int64_t sC, hipStream_t s) {
  TuneKey key{c->prec, op.M, op.K1, op.K2, batch, 10 + epi, 0, N};
  fr::GemmPlan best{op.MBW, op.NC, op.WM};
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    best = it->second;
  } else {
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    float best_ms = 1e30f;
    std::vector<fr::GemmPlan> cands = fr::gemm_candidates(op.M, batch * N, c->prec);
    sparse_candidates(op, 0, c->D, cands);
    for (const fr::GemmPlan &p : cands) {
      GemmOp trial = op;
      trial.d_A = p.MBW ? pack_upload(c, op, p, s, false) : nullptr;
      trial.MBW = p.MBW; trial.NC = p.NC; trial.WM = p.WM;
      if (p.MBW == 0) apply_sparse_plan(trial, p, c->NV);
      float ms = 0;
      try {
        for (int w = 0; w < 2; ++w) adj_gemm(c, trial, B1, B2, C, N, epi, batch, sB1, sC, s);
        hip_check(hipEventRecord(e0, s), "record");
        for (int w = 0; w < 5; ++w) adj_gemm(c, trial, B1, B2, C, N, epi, batch, sB1, sC, s);
        hip_check(hipEventRecord(e1, s), "record");
        hip_check(hipEventSynchronize(e1), "sync");
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
      } catch (...) {
        hipFree(trial.d_A);
        throw;
      }
      hipFree(trial.d_A);
      if (ms < best_ms) { best_ms = ms; best = p; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    g_tuned[key] = best;
  }
  if (best.MBW != op.MBW || best.NC != op.NC || best.WM != op.WM) {
    op.d_A = best.MBW ? pack_upload(c, op, best, s, true) : nullptr;
    op.MBW = best.MBW; op.NC = best.NC; op.WM = best.WM;
    if (best.MBW == 0) apply_sparse_plan(op, best, c->NV);
  }
}

// ulam = (dR/du)(u)^T lam, the reverse of rhs_chain
struct Primal {
  const double *uf, *qf, *q;  // U^f, Q^f, Q of the state (null: recompute)
};

// Q b += blockdiag(M0)^T Q^f b, then Q~ b = J^-1 Q b (the reverse of the
// gradient transform): one sparse-row launch with both fused where the plan
// allows it, else the product and the transform kernel.
void adj_m0t_transform(fr_ctx *c, BlockRT &b, const GemmOp &op, hipStream_t s) {
  const int D = c->D;
  const int64_t N = (int64_t)c->NV * b.ld;
  if (op.MBW == 0 && !(op.WM & kPlanStaged)) {
    fr::GemmArgs g = gemm_args(op);
    g.B1 = c->d_qfb + b.qfoff; g.ldb1 = N; g.C = c->d_ftb + b.ftoff; g.ldc = N; g.N = N;
    g.sB1 = (int64_t)b.Nf * N; g.sC = (int64_t)b.Nu * N;
    g.ld = b.ld; g.nelem = b.nelem; g.rcpdjac = b.d_rcpdjac;
    g.smat = b.d_smat; g.D = D; g.Nu = b.Nu;
    hip_check(launch_op(op, fr::PREC_F64, fr::EPI_ADDT, g, 1, s), "M0^T + J^-1");
  } else {
    adj_gemm(c, op, c->d_qfb + b.qfoff, nullptr, c->d_ftb + b.ftoff, N, fr::EPI_ADD, D,
             (int64_t)b.Nf * N, (int64_t)b.Nu * N, s);
    fr::AdjPointArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ndims = D; a.nvars = c->NV; a.nupts = b.Nu; a.ld = b.ld; a.nelem = b.nelem;
    a.smat = b.d_smat; a.rcpdjac = b.d_rcpdjac; a.fb = c->d_ftb + b.ftoff;
    hip_check(fr::launch_gradcoru_t(a, s), "gradcoru_t");
  }
}

// Tune the adjoint's M0^T product of a Navier-Stokes block together with the
// reverse gradient transform that follows it (fused or not, per plan).
void tune_adj_m0t(fr_ctx *c, BlockRT &b, hipStream_t s) {
  GemmOp &op = b.t_m0;
  const int64_t N = (int64_t)c->NV * b.ld;
  TuneKey key{c->prec, op.M, op.K1, op.K2, c->D, 20, 0, N};
  fr::GemmPlan best{op.MBW, op.NC, op.WM};
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    best = it->second;
  } else {
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    float best_ms = 1e30f;
    std::vector<fr::GemmPlan> cands = fr::gemm_candidates(op.M, c->D * N, c->prec);
    sparse_candidates(op, 0, c->D, cands);
    for (const fr::GemmPlan &p : cands) {
      if (p.MBW == 0 && (p.WM & kPlanFields) && op.sp.width > FR_SPOP_GRADT_FIELDS_WMAX) continue;
      GemmOp trial = op;
      trial.d_A = p.MBW ? pack_upload(c, op, p, s, false) : nullptr;
      trial.MBW = p.MBW; trial.NC = p.NC; trial.WM = p.WM;
      if (p.MBW == 0) apply_sparse_plan(trial, p, c->NV);
      float ms = 0;
      try {
        for (int w = 0; w < 2; ++w) adj_m0t_transform(c, b, trial, s);
        hip_check(hipEventRecord(e0, s), "record");
        for (int w = 0; w < 5; ++w) adj_m0t_transform(c, b, trial, s);
        hip_check(hipEventRecord(e1, s), "record");
        hip_check(hipEventSynchronize(e1), "sync");
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
      } catch (...) {
        hipFree(trial.d_A);
        throw;
      }
      hipFree(trial.d_A);
      if (ms < best_ms) { best_ms = ms; best = p; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    g_tuned[key] = best;
  }
  if (best.MBW != op.MBW || best.NC != op.NC || best.WM != op.WM) {
    op.d_A = best.MBW ? pack_upload(c, op, best, s, true) : nullptr;
    op.MBW = best.MBW; op.NC = best.NC; op.WM = best.WM;
    if (best.MBW == 0) apply_sparse_plan(op, best, c->NV);
  }
}

// The (M1 - M3 M2)^T product followed by the flux VJP kernel, against the
// fused plans (every field per thread, the flux VJP in the epilogue), on
// the scratch arrays; the fastest is kept (memoised per shape).
void tune_adj_tfvjp(fr_ctx *c, BlockRT &b, hipStream_t s) {
  GemmOp &op = b.t_m1;
  if (!op.sp.colidx || op.sp.width > FR_SPOP_GRADT_FIELDS_WMAX) return;
  const int64_t N = (int64_t)c->NV * b.ld;
  TuneKey key{c->prec, op.M, op.K1, op.K2, 1, 10 + fr::EPI_TFVJP, c->ns ? 1 : 0, N};
  fr::GemmPlan best{op.MBW, op.NC, op.WM};
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    best = it->second;
  } else {
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    fr::AdjPointArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ndims = c->D; a.nvars = c->NV; a.nupts = b.Nu; a.ld = b.ld; a.nelem = b.nelem;
    a.smat = b.d_smat; a.rcpdjac = b.d_rcpdjac; a.u = c->d_stage + b.uoff;
    a.q = c->ns ? (const double *)c->d_ft + b.ftoff : nullptr;
    a.fb = c->d_ftb + b.ftoff; a.ulam = c->d_w + b.uoff;
    a.gamma = c->cfg.gamma; a.mu = c->cfg.mu; a.prandtl = c->cfg.prandtl;
    std::vector<fr::GemmPlan> cands{best};
    for (int rpg : {1, 2, 4, 8, 16})
      cands.push_back(fr::GemmPlan{0, rpg, kPlanFields | kPlanFusedFluxVjp});
    float best_ms = 1e30f;
    for (const fr::GemmPlan &p : cands) {
      GemmOp trial = op;
      trial.MBW = p.MBW; trial.NC = p.NC; trial.WM = p.WM;
      if (p.MBW == 0) apply_sparse_plan(trial, p, c->NV);
      const bool fused = p.MBW == 0 && (p.WM & kPlanFusedFluxVjp);
      auto run = [&]() {
        if (fused) {
          adj_m1t_fused(c, b, trial, c->d_stage, (const double *)c->d_ft, c->d_w, s);
        } else {
          adj_gemm(c, trial, c->d_lt + b.uoff, nullptr, c->d_ftb + b.ftoff, N, fr::EPI_STORE, 1,
                   0, 0, s);
          hip_check(fr::launch_tflux_vjp(a, c->ns, s), "tflux_vjp");
        }
      };
      float ms = 0;
      for (int w = 0; w < 2; ++w) run();
      hip_check(hipEventRecord(e0, s), "record");
      for (int w = 0; w < 5; ++w) run();
      hip_check(hipEventRecord(e1, s), "record");
      hip_check(hipEventSynchronize(e1), "sync");
      hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
      if (ms < best_ms) { best_ms = ms; best = p; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    g_tuned[key] = best;
  }
  if (best.MBW != op.MBW || best.NC != op.NC || best.WM != op.WM) {
    op.d_A = best.MBW ? pack_upload(c, op, best, s, true) : nullptr;
    op.MBW = best.MBW; op.NC = best.NC; op.WM = best.WM;
    if (best.MBW == 0) apply_sparse_plan(op, best, c->NV);
  }
}

void tune_adjoint_ops(fr_ctx *c, hipStream_t s) {
  const int D = c->D, NV = c->NV;
  for (auto &b : c->blocks) {
    const int64_t N = (int64_t)NV * b.ld;
    tune_adj(c, b.t_m3, c->d_lt + b.uoff, nullptr, c->d_ufb + b.ufoff, N, fr::EPI_STORE, 1, 0, 0, s);
    tune_adj(c, b.t_m1, c->d_lt + b.uoff, nullptr, c->d_ftb + b.ftoff, N, fr::EPI_STORE, 1, 0, 0, s);
    tune_adj_tfvjp(c, b, s);
    if (c->ns) {
      tune_adj_m0t(c, b, s);
      tune_adj(c, b.t_m6, c->d_ftb + b.ftoff, nullptr, c->d_qfb + b.qfoff, N, fr::EPI_STORE, 1, 0,
               0, s);
      tune_adj(c, b.t_fin, c->d_ftb + b.ftoff, c->d_ufb + b.ufoff, c->d_w + b.uoff, N,
               fr::EPI_ADD, 1, 0, 0, s);
    } else {
      tune_adj(c, b.t_m0, c->d_ufb + b.ufoff, nullptr, c->d_w + b.uoff, N, fr::EPI_ADD, 1, 0, 0, s);
    }
  }
  hip_check(hipStreamSynchronize(s), "tune sync");
}

// The RK4 reverse update that follows a stage's right-hand-side adjoint
// (the step adjoint's bookkeeping): acc += w and, unless last, the next
// stage's scaled cotangent -J^-1 (ca dt lam + cb dt w) into c->d_lt, with
// lam = lam_{n+1} in c->d_lc.
struct RkAdj {
  const double *dt;
  double ca, cb;
  bool last;
  double *acc;
};

// lam_scaled: lam is c->d_lt already holding -J^-1 lam (written so by the
// RK adjoint bookkeeping kernel), and the scaling kernel is skipped.
// ra: the RK4 reverse update to apply to the result w = ulam, fused into
// the last product's epilogue where its plan is the sparse-row kernel.
void rhs_adjoint_chain(fr_ctx *c, const double *u, const double *lam, double *ulam,
                       hipStream_t s, Primal pr = Primal{nullptr, nullptr, nullptr},
                       bool lam_scaled = false, const RkAdj *ra = nullptr) {
  const int D = c->D, NV = c->NV;
  if (!c->adj_tuned) {
    c->adj_tuned = true;
    tune_adjoint_ops(c, s);
  }
  if (!pr.uf) {
    // primal intermediates: U^f (and C^f -> Q, Q^f for Navier-Stokes)
    rhs_chain(c, u, nullptr, fr::EPI_NEGDIV, nullptr, nullptr, s, c->ns ? 5 : 1);
    pr = Primal{(const double *)c->d_uf, (const double *)c->d_qf, (const double *)c->d_ft};
  }
  const double *ft = pr.q;
  for (auto &b : c->blocks) {
    const int64_t N = (int64_t)NV * b.ld;
    if (!lam_scaled)
      hip_check(fr::launch_negscale(NV, b.Nu, b.ld, b.nelem, b.d_rcpdjac, lam + b.uoff,
                                    c->d_lt + b.uoff, s), "negscale");
    // D~b = M3^T lt ; F~b = (M1 - M3 M2)^T lt (or, fused, the flux VJP of F~b)
    adj_gemm(c, b.t_m3, c->d_lt + b.uoff, nullptr, c->d_ufb + b.ufoff, N, fr::EPI_STORE, 1, 0, 0, s);
    if (tfvjp_fused(b))
      adj_m1t_fused(c, b, b.t_m1, u, ft, ulam, s);
    else
      adj_gemm(c, b.t_m1, c->d_lt + b.uoff, nullptr, c->d_ftb + b.ftoff, N, fr::EPI_STORE, 1, 0, 0, s);
  }
  {
    fr::AdjPairArgs pa = adj_pair_args(c);
    pa.uf = pr.uf; pa.qf = pr.qf;
    hip_check(fr::launch_comm_flux_vjp(pa, c->ns, s), "comm_flux_vjp");
  }
  for (auto &b : c->blocks) {
    fr::AdjPointArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ndims = D; a.nvars = NV; a.nupts = b.Nu; a.ld = b.ld; a.nelem = b.nelem;
    a.smat = b.d_smat; a.rcpdjac = b.d_rcpdjac; a.u = u + b.uoff; a.q = ft ? ft + b.ftoff : nullptr;
    a.fb = c->d_ftb + b.ftoff; a.ulam = ulam + b.uoff;
    a.gamma = c->cfg.gamma; a.mu = c->cfg.mu; a.prandtl = c->cfg.prandtl;
    if (!tfvjp_fused(b)) hip_check(fr::launch_tflux_vjp(a, c->ns, s), "tflux_vjp");
    const int64_t N = (int64_t)NV * b.ld;
    if (c->ns) {
      adj_m0t_transform(c, b, b.t_m0, s);
      // C^f b = M6^T Q~b (into the first rows of the Q^f b region)
      adj_gemm(c, b.t_m6, c->d_ftb + b.ftoff, nullptr, c->d_qfb + b.qfoff, N, fr::EPI_STORE, 1,
               0, 0, s);
    }
  }
  if (c->ns) hip_check(fr::launch_con_u_vjp(adj_pair_args(c), s), "con_u_vjp");
  for (auto &b : c->blocks) {
    const int64_t N = (int64_t)NV * b.ld;
    const GemmOp &fin = c->ns ? b.t_fin : b.t_m0;
    const double *B1 = c->ns ? c->d_ftb + b.ftoff : c->d_ufb + b.ufoff;
    const double *B2 = c->ns ? c->d_ufb + b.ufoff : nullptr;
    if (ra && fin.MBW == 0 && !(fin.WM & kPlanStaged)) {
      // w = ulam + the product, then the RK4 reverse update, in one pass
      fr::GemmArgs g = gemm_args(fin);
      g.B1 = B1; g.ldb1 = N; g.B2 = B2; g.ldb2 = N;
      g.C = ulam + b.uoff; g.ldc = N; g.N = N;
      g.ld = b.ld; g.nelem = b.nelem; g.rcpdjac = b.d_rcpdjac;
      g.dt = ra->dt; g.prob = b.d_prob;
      g.rk.a_next = ra->ca; g.rk.b = ra->cb; g.rk.first = 0; g.rk.last = ra->last;
      g.acc = ra->acc + b.uoff; g.stage = c->d_lc + b.uoff;
      g.out = ra->last ? nullptr : c->d_lt + b.uoff;
      hip_check(launch_op(fin, fr::PREC_F64, fr::EPI_RKADJ, g, 1, s), "adjoint gemm + RK update");
      continue;
    }
    adj_gemm(c, fin, B1, B2, ulam + b.uoff, N, fr::EPI_ADD, 1, 0, 0, s);
    if (ra)
      hip_check(fr::launch_rk_adj((int64_t)b.Nu * NV * b.ld, b.ld, b.nelem, b.d_prob, ra->dt,
                                  ra->ca, ra->cb, c->d_lc + b.uoff, ulam + b.uoff,
                                  ra->acc + b.uoff, ra->last ? nullptr : c->d_lt + b.uoff, 0,
                                  NV, b.d_rcpdjac, nullptr, s),
                "rk adjoint update");
  }
}

void axpy_blocks(fr_ctx *c, const double *dt, double coef, const double *x, const double *y,
                 double *out, hipStream_t s) {
  for (auto &b : c->blocks)
    hip_check(fr::launch_axpy_dt((int64_t)b.Nu * c->NV * b.ld, b.ld, b.nelem, b.d_prob, dt, coef,
                                 x + b.uoff, y ? y + b.uoff : nullptr, out + b.uoff, s),
              "axpy");
}

// The step adjoint's bookkeeping over every block: lam from c->d_lc, or on
// the first call from lam_np1 (copied into c->d_lc on the way); kb goes
// to c->d_lt scaled by -1/J, ready for the next right-hand-side adjoint.
void rk_adj_blocks(fr_ctx *c, const double *dt, double ca, double cb, double *acc, int first,
                   bool last, hipStream_t s, const double *lam_np1 = nullptr) {
  for (auto &b : c->blocks)
    hip_check(fr::launch_rk_adj((int64_t)b.Nu * c->NV * b.ld, b.ld, b.nelem, b.d_prob, dt, ca, cb,
                                (lam_np1 ? lam_np1 : c->d_lc) + b.uoff, c->d_w + b.uoff,
                                acc + b.uoff, last ? nullptr : c->d_lt + b.uoff, first, c->NV,
                                b.d_rcpdjac, lam_np1 ? c->d_lc + b.uoff : nullptr, s),
              "rk adjoint update");
}

// lam_n = (d u_{n+1} / d u_n)^T lam_np1 for one classical RK4 step
void rk4_step_adjoint(fr_ctx *c, const double *u, const double *dt, const double *lam_np1,
                      double *lam_n, hipStream_t s) {
  ensure_adjoint(c, s);
  // stage states u2 = u + dt/2 k1, u3 = u + dt/2 k2, u4 = u + dt k3
  static const double a[3] = {0.5, 0.5, 1.0};
  const double *prev = u;
  for (int i = 0; i < 3; ++i) {
    rhs_chain(c, prev, c->d_k, fr::EPI_NEGDIV, nullptr, nullptr, s);
    axpy_blocks(c, dt, a[i], u, c->d_k, c->d_st[i], s);
    prev = c->d_st[i];
  }
  // acc = lam; kb = dt/6 lam ; then per stage (from the last): w = J(u_s)^T kb,
  // acc += w, kb = b_{s-1} dt lam + a_s dt w
  rk_adj_blocks(c, dt, 1.0 / 6, 0.0, lam_n, 1, false, s, lam_np1);
  const double *stages[4] = {c->d_st[2], c->d_st[1], c->d_st[0], u};
  static const double ca[3] = {1.0 / 3, 1.0 / 3, 1.0 / 6};
  static const double cb[3] = {1.0, 0.5, 0.5};
  for (int i = 0; i < 4; ++i) {
    const RkAdj ra{dt, i < 3 ? ca[i] : 0.0, i < 3 ? cb[i] : 0.0, i == 3, lam_n};
    rhs_adjoint_chain(c, stages[i], c->d_lt, c->d_w, s, Primal{nullptr, nullptr, nullptr}, true,
                      &ra);
  }
}

// Layout of one step's stash: for each stage s = 0..3 its input state, then
// (FP64) U^f, Q^f and Q of that state (the last two for Navier-Stokes only).
int64_t stash_stage_len(const fr_ctx *c) {
  return c->total_len + c->uf_len + (c->ns ? c->qf_len + c->ft_len : 0);
}

struct StashStage {
  double *state, *uf, *qf, *q;
};

StashStage stash_stage(const fr_ctx *c, double *stash, int st) {
  double *p = stash + st * stash_stage_len(c);
  StashStage r;
  r.state = p; p += c->total_len;
  r.uf = p; p += c->uf_len;
  r.qf = c->ns ? p : nullptr; if (c->ns) p += c->qf_len;
  r.q = c->ns ? p : nullptr;
  return r;
}

// One RK4 step of u in place that leaves every stage state and its primal
// intermediates in `stash` (out-of-place flux outputs keep them intact).
void rk4_step_stash(fr_ctx *c, double *u, const double *dt, double *stash, hipStream_t s) {
  static const double a_next[4] = {0.5, 0.5, 1.0, 0.0};
  static const double bw[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
  const fr_ctx::Bufs saved = c->cur;
  try {
    hip_check(hipMemcpyAsync(stash_stage(c, stash, 0).state, u, c->total_len * sizeof(double),
                             hipMemcpyDeviceToDevice, s), "copy");
    for (int st = 0; st < 4; ++st) {
      StashStage S = stash_stage(c, stash, st);
      c->cur = fr_ctx::Bufs{S.uf, c->ns ? (void *)S.qf : c->d_qf, c->ns ? (void *)S.q : c->d_ft,
                            c->d_uf, c->d_ft, st < 3 ? stash_stage(c, stash, st + 1).state : nullptr};
      fr::RkCoef rk;
      rk.a_next = a_next[st]; rk.b = bw[st]; rk.first = st == 0; rk.last = st == 3;
      rhs_chain(c, S.state, u, fr::EPI_RK, &rk, dt, s);
    }
  } catch (...) {
    c->cur = saved;
    throw;
  }
  c->cur = saved;
}

void rk4_step_adjoint_stash(fr_ctx *c, double *stash, const double *dt, const double *lam_np1,
                            double *lam_n, hipStream_t s) {
  ensure_adjoint(c, s);
  rk_adj_blocks(c, dt, 1.0 / 6, 0.0, lam_n, 1, false, s, lam_np1);
  static const double ca[3] = {1.0 / 3, 1.0 / 3, 1.0 / 6};
  static const double cb[3] = {1.0, 0.5, 0.5};
  for (int i = 0; i < 4; ++i) {
    StashStage S = stash_stage(c, stash, 3 - i);
    const RkAdj ra{dt, i < 3 ? ca[i] : 0.0, i < 3 ? cb[i] : 0.0, i == 3, lam_n};
    rhs_adjoint_chain(c, S.state, c->d_lt, c->d_w, s, Primal{S.uf, S.qf, S.q}, true, &ra);
  }
}

// Adjoint of a checkpoint segment: replay nsteps RK4 steps from u0 (into
// the context's replay state) stashing every step, then the step adjoints
// from the last step to the first: lam0 = (d u_{n0+nsteps} / d u_{n0})^T lam_end.
void rk4_segment_adjoint(fr_ctx *c, const double *u0, const double *dt, int nsteps,
                         const double *lam_end, double *lam0, double *stash, hipStream_t s) {
  const int64_t L = 4 * stash_stage_len(c);
  const size_t bytes = c->total_len * sizeof(double);
  if (nsteps == 0) {
    if (lam0 != lam_end)
      hip_check(hipMemcpyAsync(lam0, lam_end, bytes, hipMemcpyDeviceToDevice, s), "copy");
    return;
  }
  hip_check(hipMemcpyAsync(c->d_seg_u, u0, bytes, hipMemcpyDeviceToDevice, s), "copy");
  for (int i = 0; i < nsteps; ++i) rk4_step_stash(c, c->d_seg_u, dt, stash + i * L, s);
  for (int i = nsteps - 1; i >= 0; --i)
    rk4_step_adjoint_stash(c, stash + i * L, dt, i == nsteps - 1 ? lam_end : lam0, lam0, s);
}

// One classical RK4 step of u in place: k_s = R(stage_s), with
// acc = u + dt/6 k1 + dt/3 k2 + dt/3 k3 and u <- acc + dt/6 k4.
void rk4_step(fr_ctx *c, double *u, const double *dt, hipStream_t s) {
  static const double a_next[4] = {0.5, 0.5, 1.0, 0.0};
  static const double b[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
  for (int st = 0; st < 4; ++st) {
    fr::RkCoef rk;
    rk.a_next = a_next[st]; rk.b = b[st]; rk.first = st == 0; rk.last = st == 3;
    rhs_chain(c, st == 0 ? u : c->d_stage, u, fr::EPI_RK, &rk, dt, s);
  }
}

void release_graph_pair(hipGraph_t &g, hipGraphExec_t &e) {
  if (e) hipGraphExecDestroy(e);
  if (g) hipGraphDestroy(g);
  e = nullptr; g = nullptr;
}

void release_graph(fr_ctx *c) {
  release_graph_pair(c->graph, c->graph_exec);
  release_graph_pair(c->graph_k, c->graph_k_exec);
  c->graph_u = nullptr; c->graph_dt = nullptr;
}

void release_euler_graphs(fr_ctx *c) {
  release_graph_pair(c->eu_graph, c->eu_exec);
  release_graph_pair(c->eu_graph_k, c->eu_exec_k);
  c->eu_u = nullptr; c->eu_dt = nullptr;
}

void release_stepper_graphs(fr_ctx *c) {
  release_euler_graphs(c);
  if (c->dp_exec) hipGraphExecDestroy(c->dp_exec);
  if (c->dp_graph) hipGraphDestroy(c->dp_graph);
  c->dp_exec = nullptr; c->dp_graph = nullptr; c->dp_key = fr_ctx::DpKey{};
  for (auto &g : c->seg_graphs) release_graph_pair(g.graph, g.exec);
  c->seg_graphs.clear();
}

// Steps captured into one graph when a call asks for that many or more.
constexpr int kStepsPerGraph = 8;

// Capture `body` on the context's capture stream into (graph, exec).
template <typename F>
void capture(fr_ctx *c, hipGraph_t &graph, hipGraphExec_t &exec, F body) {
  hip_check(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "capture");
  try {
    body(c->cap_stream);
  } catch (...) {
    hipGraph_t g = nullptr;
    hipStreamEndCapture(c->cap_stream, &g);
    if (g) hipGraphDestroy(g);
    throw;
  }
  hip_check(hipStreamEndCapture(c->cap_stream, &graph), "end capture");
  hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
}

// One forward Euler step in place: the last-stage RK epilogue with b = 1 and
// the state itself as the register (u <- u + dt R(u)).
void euler_step(fr_ctx *c, double *u, const double *dt, hipStream_t s) {
  fr::RkCoef rk;
  rk.a_next = 0.0; rk.b = 1.0; rk.first = 1; rk.last = 1;
  const fr_ctx::Bufs saved = c->cur;
  c->cur.acc = u;
  try {
    rhs_chain(c, u, u, fr::EPI_RK, &rk, dt, s);
  } catch (...) {
    c->cur = saved;
    throw;
  }
  c->cur = saved;
}

// Dormand-Prince 5(4): stage matrix (lower triangle), and the error weights
// b - bhat of the fifth- and embedded fourth-order solutions (Dormand and
// Prince 1980).  The seventh stage is taken at the new state (its row is b).
const double kDpA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
const double kDpBhat[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                           -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

void ensure_dopri(fr_ctx *c, hipStream_t s) {
  if (c->dp_ready) return;
  for (auto &k : c->d_dpk) k = dev_alloc<double>(c, c->total_len);
  c->d_dpy = dev_alloc<double>(c, c->total_len);
  c->d_dp_ssq = dev_alloc<double>(c, c->nproblems);
  c->d_dp_ndof = dev_upload(c, c->ndof_host.data(), c->ndof_host.size(), s);
  c->d_dp_acc = dev_alloc<int32_t>(c, c->nproblems);
  c->d_dp_rej = dev_alloc<int32_t>(c, c->nproblems);
  c->dp_ready = true;
}

// One attempt on every problem: stages 2..7 (y_i = u + h sum_j a_ij k_j,
// k_i = R(y_i)), the error norms, the controller and the commit.  k1 = R(u)
// on entry; y ends as the fifth-order solution.
void dopri_attempt(fr_ctx *c, double *u, double *t, double *dt, const double *tend,
                   int32_t *counts, double atol, double rtol, hipStream_t s) {
  double *const *k = c->d_dpk;
  for (int i = 1; i < 7; ++i) {
    for (auto &b : c->blocks) {
      fr::DpStage st{};
      for (int j = 0; j < i; ++j) {
        st.a[j] = kDpA[i][j];
        st.k[j] = k[j] + b.uoff;
      }
      hip_check(fr::launch_dp_stage(i, (int64_t)b.Nu * c->NV * b.ld, b.ld, b.nelem, b.d_prob, dt,
                                    st, u + b.uoff, c->d_dpy + b.uoff, s),
                "dopri5 stage");
    }
    rhs_chain(c, c->d_dpy, k[i], fr::EPI_NEGDIV, nullptr, nullptr, s);
  }
  for (auto &b : c->blocks) {
    fr::DpError er{};
    for (int j = 0; j < 7; ++j) {
      er.E[j] = (j < 6 ? kDpA[6][j] : 0.0) - kDpBhat[j];
      er.k[j] = er.E[j] != 0.0 ? k[j] + b.uoff : nullptr;
    }
    er.atol = atol; er.rtol = rtol;
    hip_check(fr::launch_dp_error(c->NV, b.Nu, b.ld, b.nelem, c->nchunk, c->nelem_total,
                                  b.d_prob, dt, er, u + b.uoff, c->d_dpy + b.uoff,
                                  c->d_part + b.part_off, s),
              "dopri5 error");
  }
  hip_check(fr::launch_problem_sums(1, c->nproblems, c->nchunk, c->nelem_total, c->nslice,
                                    c->slice_len, c->d_pstart, c->d_plist, c->d_part, c->d_part2,
                                    c->d_dp_ssq, s),
            "dopri5 error sums");
  hip_check(fr::launch_dp_control(c->nproblems, c->d_dp_ssq, c->d_dp_ndof, t, dt, tend,
                                  c->d_dp_acc, c->d_dp_rej, counts, s),
            "dopri5 control");
  for (auto &b : c->blocks)
    hip_check(fr::launch_dp_commit((int64_t)b.Nu * c->NV * b.ld, b.ld, b.nelem, b.d_prob,
                                   c->d_dp_acc, c->d_dpy + b.uoff, k[6] + b.uoff, u + b.uoff,
                                   k[0] + b.uoff, s),
              "dopri5 commit");
}

}  // namespace

extern "C" {

fr_status fr_setup_mesh(const fr_config *cfg, int32_t nblocks, const fr_block *blocks,
                        int64_t npairs, const fr_facepair *pairs, void *hip_stream,
                        fr_ctx **out) {
  return fr_setup_mesh_bc(cfg, nblocks, blocks, npairs, pairs, 0, nullptr, 0, nullptr, hip_stream,
                          out);
}

fr_status fr_setup_mesh_bc(const fr_config *cfg, int32_t nblocks, const fr_block *blocks,
                           int64_t npairs, const fr_facepair *pairs, int32_t nbcs,
                           const fr_bc *bcs, int64_t nbcfaces, const fr_bcface *bcfaces,
                           void *hip_stream, fr_ctx **out) {
  if (!out) return fail(nullptr, FR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg || !blocks || nblocks < 1 || npairs < 0 || (npairs > 0 && !pairs))
    return fail(nullptr, FR_EINVAL, "bad arguments");
  if (nbcs < 0 || nbcfaces < 0 || (nbcs > 0 && !bcs) || (nbcfaces > 0 && !bcfaces))
    return fail(nullptr, FR_EINVAL, "bad boundary arguments");
  for (int32_t k = 0; k < nbcs; ++k)
    if (bcs[k].type < FR_BC_SUPERSONIC_INFLOW || bcs[k].type > FR_BC_NOSLIP_ISOTHERMAL_WALL)
      return fail(nullptr, FR_EINVAL, "bad boundary condition type");
  if (cfg->ndims != 2 && cfg->ndims != 3) return fail(nullptr, FR_EINVAL, "ndims must be 2 or 3");
  if (cfg->system != FR_EULER && cfg->system != FR_NAVIER_STOKES)
    return fail(nullptr, FR_EINVAL, "bad system");
  if (cfg->prec != FR_FP64 && cfg->prec != FR_FP32 && cfg->prec != FR_BF16X3)
    return fail(nullptr, FR_EUNSUPPORTED, "precision mode not available");
  if (!(cfg->gamma > 1.0)) return fail(nullptr, FR_EINVAL, "gamma must exceed 1");
  if (cfg->system == FR_NAVIER_STOKES && !(cfg->mu >= 0 && cfg->prandtl > 0))
    return fail(nullptr, FR_EINVAL, "bad viscosity or Prandtl number");
  std::unique_ptr<fr_ctx> c(new fr_ctx);
  c->cfg = *cfg;
  c->D = cfg->ndims; c->NV = cfg->ndims + 2;
  c->ns = cfg->system == FR_NAVIER_STOKES;
  c->prec = cfg->prec;
  c->tsize = cfg->prec == FR_FP64 ? 8 : 4;
  c->nproblems = cfg->nproblems > 0 ? cfg->nproblems : 1;
  hipStream_t s = (hipStream_t)hip_stream;
  const int D = c->D, NV = c->NV;
  try {
    std::map<std::tuple<int, int, int>, int> refmap;
    std::vector<fr::BlockGeom> geoms;
    std::vector<int> block_ref;
    int64_t uoff = 0, ufoff = 0, qfoff = 0, ftoff = 0, poff = 0, refoff = 0;
    for (int bi = 0; bi < nblocks; ++bi) {
      const fr_block &B = blocks[bi];
      if (B.nelem < 1 || !B.nodes) throw Fail{FR_EINVAL, "block without elements or nodes"};
      if (block_too_large(B, NV)) throw Fail{FR_EINVAL, kBlockTooLarge};
      if ((B.etype == FR_HEX) != (D == 3) || B.etype < 0 || B.etype > 2)
        throw Fail{FR_EINVAL, "element type does not match ndims"};
      auto key = std::make_tuple(B.etype, B.order, B.correction);
      if (!refmap.count(key)) {
        refmap[key] = (int)c->refs.size();
        c->refs.push_back(fr::build_ref(B.etype, B.order, B.correction));
      }
      BlockRT rt;
      rt.ref = refmap[key];
      const fr::RefOps &R = c->refs[rt.ref];
      rt.etype = B.etype; rt.order = B.order;
      rt.nelem = B.nelem; rt.ld = round_up(B.nelem, 16);
      rt.Nu = R.nupts; rt.Nf = R.nfpts;
      geoms.push_back(fr::build_geom(R, B.geom_order, B.nelem, B.nodes, rt.ld));
      block_ref.push_back(rt.ref);
      rt.uoff = uoff; uoff += (int64_t)rt.Nu * NV * rt.ld;
      rt.ufoff = ufoff; ufoff += (int64_t)rt.Nf * NV * rt.ld;
      rt.qfoff = qfoff; qfoff += (int64_t)D * rt.Nf * NV * rt.ld;
      rt.ftoff = ftoff; ftoff += (int64_t)D * rt.Nu * NV * rt.ld;
      rt.part_off = poff; poff += B.nelem;
      rt.refoff = refoff; refoff += (int64_t)NV * rt.ld;
      c->blocks.push_back(std::move(rt));
    }
    c->total_len = uoff; c->uf_len = ufoff; c->qf_len = c->ns ? qfoff : 0; c->ft_len = ftoff;
    c->nelem_total = poff;
    if (ufoff >= (1ll << 31) || qfoff >= (1ll << 31))
      throw Fail{FR_EUNSUPPORTED, "mesh too large for 32-bit flux-point indices"};
    // pairs
    std::vector<fr::FacePairIn> pin(npairs);
    for (int64_t k = 0; k < npairs; ++k) {
      const fr_facepair &P = pairs[k];
      pin[k] = fr::FacePairIn{P.lblock, P.lface, P.lelem, P.rblock, P.rface, P.relem,
                              {P.shift[0], P.shift[1], P.shift[2]}};
    }
    std::vector<fr::BcFaceIn> bin(nbcfaces);
    for (int64_t k = 0; k < nbcfaces; ++k)
      bin[k] = fr::BcFaceIn{bcfaces[k].block, bcfaces[k].face, bcfaces[k].elem, bcfaces[k].bc};
    fr::BcTable BT;
    fr::PairTable T = fr::build_pairs(c->refs, geoms, block_ref, D, NV, pin.data(), npairs,
                                      bin.data(), nbcfaces, nbcs, &BT);
    c->npairs = T.n;
    c->nbpts = BT.n;
    if (BT.n) {
      std::vector<int32_t> bi(BT.n);
      for (int64_t i = 0; i < BT.n; ++i) bi[i] = (int32_t)BT.idx[i];
      c->d_bidx = dev_upload(c.get(), bi.data(), BT.n, s);
      c->d_bblk = dev_upload(c.get(), BT.blk.data(), BT.n, s);
      c->d_bcid = dev_upload(c.get(), BT.bc.data(), BT.n, s);
      c->d_bnrm = dev_upload(c.get(), BT.nrm.data(), BT.nrm.size(), s);
      c->d_bmag = dev_upload(c.get(), BT.mag.data(), BT.n, s);
      std::vector<double> par((size_t)nbcs * FR_BC_NPAR, 0.0);
      for (int32_t k = 0; k < nbcs; ++k) {
        double *q = &par[(size_t)k * FR_BC_NPAR];
        q[0] = bcs[k].type; q[1] = bcs[k].rho;
        for (int d = 0; d < 3; ++d) { q[2 + d] = bcs[k].v[d]; q[7 + d] = bcs[k].vw[d]; }
        q[5] = bcs[k].p; q[6] = bcs[k].cp_tw;
      }
      c->d_bcpar = dev_upload(c.get(), par.data(), par.size(), s);
    }
    // device data: geometry and operators
    for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
      BlockRT &b = c->blocks[bi];
      fr::BlockGeom &G = geoms[bi];
      const fr::RefOps &R = c->refs[b.ref];
      b.d_smat = dev_upload(c.get(), G.smat.data(), G.smat.size(), s);
      b.d_rcpdjac = dev_upload(c.get(), G.rcpdjac.data(), G.rcpdjac.size(), s);
      b.d_wdjac = dev_upload(c.get(), G.wdjac.data(), G.wdjac.size(), s);
      b.xu = std::move(G.xu);
      b.wdjac_host.resize((size_t)b.Nu * b.nelem);
      for (int r = 0; r < b.Nu; ++r)
        for (int64_t n = 0; n < b.nelem; ++n)
          b.wdjac_host[(size_t)r * b.nelem + n] = G.wdjac[(size_t)r * b.ld + n];
      if (blocks[bi].problem) {
        for (int64_t n = 0; n < b.nelem; ++n)
          if (blocks[bi].problem[n] < 0 || blocks[bi].problem[n] >= c->nproblems)
            throw Fail{FR_EINVAL, "problem id out of range"};
        b.d_prob = dev_upload(c.get(), blocks[bi].problem, b.nelem, s);
      }
      const int64_t N = (int64_t)NV * b.ld;
      // LDS chunk hints: the flux points of one face, one direction of F~
      const int nface = b.etype == 0 ? 4 : b.etype == 1 ? 3 : 6;
      make_op(c.get(), b.m0, R.M0, R.nfpts, R.nupts, 0, N, s);
      make_op(c.get(), b.s8, hcat(R.M3, R.nfpts, R.M1p, D * R.nupts, R.nupts), R.nupts,
              R.nfpts, D * R.nupts, N, s, nullptr, R.nfpts / nface, R.nupts);
      if (c->ns) {
        make_op(c.get(), b.s3, hcat(R.M6, R.nfpts, R.M4p, R.nupts, D * R.nupts), D * R.nupts,
                R.nfpts, R.nupts, N, s, nullptr, R.nfpts / nface);
        make_op(c.get(), b.m5, R.M0, R.nfpts, R.nupts, 0, D * N, s);
      }
      G = fr::BlockGeom();
    }
    // pair table
    {
      std::vector<int32_t> li(T.n), ri(T.n);
      for (int64_t i = 0; i < T.n; ++i) { li[i] = (int32_t)T.lidx[i]; ri[i] = (int32_t)T.ridx[i]; }
      c->d_lidx = dev_upload(c.get(), li.data(), T.n, s);
      c->d_ridx = dev_upload(c.get(), ri.data(), T.n, s);
      c->d_lblk = dev_upload(c.get(), T.lblk.data(), T.n, s);
      c->d_rblk = dev_upload(c.get(), T.rblk.data(), T.n, s);
      c->d_nrm = dev_upload(c.get(), T.nrm.data(), T.nrm.size(), s);
      c->d_magL = dev_upload(c.get(), T.magL.data(), T.n, s);
      c->d_magR = dev_upload(c.get(), T.magR.data(), T.n, s);
      std::vector<int64_t> ub, qb, lds, qs;
      for (auto &b : c->blocks) {
        ub.push_back(b.ufoff); qb.push_back(b.qfoff); lds.push_back(b.ld);
        qs.push_back((int64_t)b.Nf * NV * b.ld);
      }
      c->d_blk_ufbase = dev_upload(c.get(), ub.data(), ub.size(), s);
      c->d_blk_qfbase = dev_upload(c.get(), qb.data(), qb.size(), s);
      c->d_blk_ld = dev_upload(c.get(), lds.data(), lds.size(), s);
      c->d_blk_qstride = dev_upload(c.get(), qs.data(), qs.size(), s);
    }
    // scratch
    // U^f (then D~) and F~ in one allocation, so that the divergence
    // product's two panels lie within one 32-bit buffer range (precomputed
    // row offsets) on meshes up to a few GiB of them
    {
      const int64_t al = 256 / (int64_t)c->tsize;  // 256-byte aligned parts
      const int64_t nuf = (c->uf_len + al - 1) / al * al, nft = (c->ft_len + al - 1) / al * al;
      const int64_t tot = nuf + nft + (c->ns ? nft : 0);
      char *arena = c->prec == FR_FP64 ? (char *)dev_alloc<double>(c.get(), tot)
                                       : (char *)dev_alloc<float>(c.get(), tot);
      c->d_uf = arena;
      c->d_ft = arena + nuf * c->tsize;
      if (c->ns) c->d_fto = arena + (nuf + nft) * c->tsize;
    }
    if (c->ns)
      c->d_qf = c->prec == FR_FP64 ? (void *)dev_alloc<double>(c.get(), c->qf_len)
                                    : (void *)dev_alloc<float>(c.get(), c->qf_len);
    c->d_acc = dev_alloc<double>(c.get(), c->total_len);
    c->d_stage = dev_alloc<double>(c.get(), c->total_len);
    c->devform = c->prec != FR_FP64;
    if (c->devform) {
      c->d_udev = dev_alloc<float>(c.get(), c->total_len);
      int64_t nref = 0;
      std::vector<int64_t> rb;
      for (auto &b : c->blocks) { rb.push_back(b.refoff); nref += (int64_t)NV * b.ld; }
      c->d_uref = dev_alloc<double>(c.get(), nref);
      c->d_blk_refbase = dev_upload(c.get(), rb.data(), rb.size(), s);
    }
    c->cur = fr_ctx::Bufs{c->d_uf, c->d_qf, c->d_ft, c->d_uf, c->ns ? c->d_fto : c->d_ft,
                          c->d_stage};
    // precomputed row offsets of the sparse-row products of steps 1, 5 and 8
    // (per block, and the multi-block launches' slots)
    for (auto &b : c->blocks) {
      const int64_t rsu = (int64_t)NV * b.ld * 8, rst = (int64_t)NV * b.ld * (int64_t)c->tsize;
      // step 1 reads the state, or in the deviation form its FP32 deviation
      const int64_t rs0 = c->devform ? rst : rsu;
      build_row_offsets(c.get(), b.m0, nullptr, rs0, nullptr, 0, rs0, s);
      if (c->ns) build_row_offsets(c.get(), b.m5, nullptr, rst, nullptr, 0, rst, s);
      build_row_offsets(c.get(), b.s8, elem(c->cur.df, b.ufoff, c->tsize), rst,
                        elem(c->cur.fto, b.ftoff, c->tsize), rst, rst, s);
    }
    // reductions: element partials and per-problem element lists
    {
      // enough workgroups to fill the chip on small meshes
      int64_t wgs = 0;
      for (auto &b : c->blocks) wgs += (b.nelem + 63) / 64;
      c->nchunk = (int)std::min<int64_t>(16, std::max<int64_t>(1, 2048 / std::max<int64_t>(1, wgs)));
    }
    c->d_part = dev_alloc<double>(c.get(), (size_t)c->nchunk * c->nelem_total * (NV + 1));
    {
      std::vector<std::vector<int64_t>> lists(c->nproblems);
      c->ndof_host.assign(c->nproblems, 0.0);
      for (size_t bi = 0; bi < c->blocks.size(); ++bi)
        for (int64_t n = 0; n < c->blocks[bi].nelem; ++n) {
          int pr = blocks[bi].problem ? blocks[bi].problem[n] : 0;
          lists[pr].push_back(c->blocks[bi].part_off + n);
          c->ndof_host[pr] += (double)c->blocks[bi].Nu * NV;
        }
      std::vector<int64_t> start(1, 0), flat;
      size_t maxlen = 0;
      for (auto &l : lists) {
        flat.insert(flat.end(), l.begin(), l.end());
        start.push_back(flat.size());
        maxlen = std::max(maxlen, l.size());
      }
      // 64 list entries per slice, more once there would be over 32768 slices
      const int64_t blocks64 = std::max<int64_t>(1, ((int64_t)maxlen + 63) / 64);
      c->slice_len = 64 * ((blocks64 + 32767) / 32768);
      c->nslice = (int)std::max<int64_t>(1, ((int64_t)maxlen + c->slice_len - 1) / c->slice_len);
      if (c->nslice > 1)
        c->d_part2 = dev_alloc<double>(c.get(), (size_t)c->nproblems * c->nslice * (NV + 1));
      c->d_pstart = dev_upload(c.get(), start.data(), start.size(), s);
      c->d_plist = dev_upload(c.get(), flat.data(), flat.size(), s);
    }
    c->d_flag = dev_alloc<int32_t>(c.get(), 1);
    {
      // indexed by problem id in the RK epilogue
      const std::vector<double> zeros((size_t)c->nproblems, 0.0);
      c->d_tune_dt = dev_upload(c.get(), zeros.data(), zeros.size(), s);
    }
    if (cfg->autotune) autotune(c.get(), s);
    {
      // the integrals' fixed scratch of this device (fr_integrate_noalloc)
      double *scr = nullptr;
      hip_check(fr::integral_scratch(&scr), "integral scratch address");
    }
    hip_check(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "stream");
    hip_check(hipDeviceSynchronize(), "setup sync");
  } catch (const fr::SetupError &e) {
    fr_destroy(c.release());
    return fail(nullptr, (fr_status)e.status, e.what());
  } catch (const Fail &f) {
    fr_destroy(c.release());
    return fail(nullptr, f.st, f.msg);
  } catch (const std::exception &e) {
    fr_destroy(c.release());
    return fail(nullptr, FR_ENOMEM, e.what());
  }
  *out = c.release();
  return FR_OK;
}

fr_status fr_get_layout(const fr_ctx *c, int32_t block, int64_t *offset, int64_t *ld,
                        int32_t *nupts, int32_t *nvars, int64_t *total_len) {
  if (!c || block < 0 || block >= (int)c->blocks.size()) return FR_EINVAL;
  const BlockRT &b = c->blocks[block];
  if (offset) *offset = b.uoff;
  if (ld) *ld = b.ld;
  if (nupts) *nupts = b.Nu;
  if (nvars) *nvars = c->NV;
  if (total_len) *total_len = c->total_len;
  return FR_OK;
}

fr_status fr_get_solution_points(const fr_ctx *c, int32_t block, double *xyz) {
  if (!c || !xyz || block < 0 || block >= (int)c->blocks.size()) return FR_EINVAL;
  const BlockRT &b = c->blocks[block];
  std::memcpy(xyz, b.xu.data(), b.xu.size() * sizeof(double));
  return FR_OK;
}

fr_status fr_get_quadrature(const fr_ctx *c, int32_t block, double *wj) {
  if (!c || !wj || block < 0 || block >= (int)c->blocks.size()) return FR_EINVAL;
  const BlockRT &b = c->blocks[block];
  std::memcpy(wj, b.wdjac_host.data(), b.wdjac_host.size() * sizeof(double));
  return FR_OK;
}

fr_status fr_rhs(fr_ctx *c, const double *u, double *dudt, void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !dudt) return fail(c, FR_EINVAL, "null state pointer");
  try {
    rhs_chain(c, u, dudt, fr::EPI_NEGDIV, nullptr, nullptr, (hipStream_t)hip_stream);
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_rk_step(fr_ctx *c, double *u, const double *dt_dev, int32_t nsteps,
                     void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !dt_dev || nsteps < 0) return fail(c, FR_EINVAL, "bad rk_step arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    if (nsteps > 0 && (c->graph_u != u || c->graph_dt != dt_dev)) {
      release_graph(c);
      c->graph_u = u; c->graph_dt = dt_dev;
    }
    // groups of kStepsPerGraph steps in one graph (one launch gap per group),
    // the rest one step per launch: the same kernels in the same order
    int done = 0;
    if (nsteps >= kStepsPerGraph) {
      if (!c->graph_k_exec)
        capture(c, c->graph_k, c->graph_k_exec, [&](hipStream_t cs) {
          for (int k = 0; k < kStepsPerGraph; ++k) rk4_step(c, u, dt_dev, cs);
        });
      for (; done + kStepsPerGraph <= nsteps; done += kStepsPerGraph)
        hip_check(hipGraphLaunch(c->graph_k_exec, s), "graph launch");
    }
    if (done < nsteps && !c->graph_exec)
      capture(c, c->graph, c->graph_exec, [&](hipStream_t cs) { rk4_step(c, u, dt_dev, cs); });
    for (; done < nsteps; ++done) hip_check(hipGraphLaunch(c->graph_exec, s), "graph launch");
    if (c->cfg.check_finite) {
      int32_t h = 0;
      hip_check(hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), s), "memset");
      hip_check(fr::launch_check_finite(u, c->total_len, c->d_flag, s), "check_finite");
      hip_check(hipMemcpyAsync(&h, c->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
      hip_check(hipStreamSynchronize(s), "sync");
      if (h) return fail(c, FR_ENONFINITE, "state contains NaN or Inf");
    }
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_euler_step(fr_ctx *c, double *u, const double *dt_dev, int32_t nsteps,
                        void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !dt_dev || nsteps < 0) return fail(c, FR_EINVAL, "bad euler_step arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    if (nsteps > 0 && (c->eu_u != u || c->eu_dt != dt_dev)) {
      release_euler_graphs(c);
      c->eu_u = u; c->eu_dt = dt_dev;
    }
    int done = 0;
    if (nsteps >= kStepsPerGraph) {
      if (!c->eu_exec_k)
        capture(c, c->eu_graph_k, c->eu_exec_k, [&](hipStream_t cs) {
          for (int k = 0; k < kStepsPerGraph; ++k) euler_step(c, u, dt_dev, cs);
        });
      for (; done + kStepsPerGraph <= nsteps; done += kStepsPerGraph)
        hip_check(hipGraphLaunch(c->eu_exec_k, s), "graph launch");
    }
    if (done < nsteps && !c->eu_exec)
      capture(c, c->eu_graph, c->eu_exec, [&](hipStream_t cs) { euler_step(c, u, dt_dev, cs); });
    for (; done < nsteps; ++done) hip_check(hipGraphLaunch(c->eu_exec, s), "graph launch");
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_dopri5_step(fr_ctx *c, double *u, double *t, double *dt, const double *tend,
                         int32_t nattempts, double atol, double rtol, int32_t *counts,
                         void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !t || !dt || nattempts < 0) return fail(c, FR_EINVAL, "bad dopri5_step arguments");
  if (!(atol > 0) || !(rtol > 0) || !std::isfinite(atol) || !std::isfinite(rtol))
    return fail(c, FR_EINVAL, "tolerances must be positive and finite");
  if (nattempts == 0) return FR_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    ensure_dopri(c, s);
    const fr_ctx::DpKey key{u, t, dt, tend, counts, atol, rtol};
    if (!c->dp_exec || !(c->dp_key == key)) {
      if (c->dp_exec) hipGraphExecDestroy(c->dp_exec);
      if (c->dp_graph) hipGraphDestroy(c->dp_graph);
      c->dp_exec = nullptr; c->dp_graph = nullptr;
      capture(c, c->dp_graph, c->dp_exec, [&](hipStream_t cs) {
        dopri_attempt(c, u, t, dt, tend, counts, atol, rtol, cs);
      });
      c->dp_key = key;
    }
    hip_check(fr::launch_dp_clamp(c->nproblems, t, tend, dt, s), "dopri5 clamp");
    rhs_chain(c, u, c->d_dpk[0], fr::EPI_NEGDIV, nullptr, nullptr, s);
    for (int i = 0; i < nattempts; ++i) hip_check(hipGraphLaunch(c->dp_exec, s), "graph launch");
    if (c->cfg.check_finite) {
      int32_t h = 0;
      hip_check(hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), s), "memset");
      hip_check(fr::launch_check_finite(u, c->total_len, c->d_flag, s), "check_finite");
      hip_check(hipMemcpyAsync(&h, c->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
      hip_check(hipStreamSynchronize(s), "sync");
      if (h) return fail(c, FR_ENONFINITE, "state contains NaN or Inf");
    }
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_rhs_adjoint(fr_ctx *c, const double *u, const double *lam, double *ulam,
                         void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !lam || !ulam || ulam == u || ulam == lam)
    return fail(c, FR_EINVAL, "bad adjoint arguments (ulam must not alias u or lam)");
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    ensure_adjoint(c, s);
    rhs_adjoint_chain(c, u, lam, ulam, s);
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_rk_step_adjoint(fr_ctx *c, const double *u_n, const double *dt_dev,
                             const double *lam_np1, double *lam_n, void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u_n || !dt_dev || !lam_np1 || !lam_n || lam_n == u_n)
    return fail(c, FR_EINVAL, "bad step adjoint arguments");
  try {
    rk4_step_adjoint(c, u_n, dt_dev, lam_np1, lam_n, (hipStream_t)hip_stream);
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_stash_len(const fr_ctx *c, int64_t *len) {
  if (!c || !len) return FR_EINVAL;
  *len = 4 * stash_stage_len(c);
  return FR_OK;
}

fr_status fr_rk_step_stash(fr_ctx *c, double *u, const double *dt_dev, double *stash,
                           void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !dt_dev || !stash) return fail(c, FR_EINVAL, "bad stash step arguments");
  if (c->prec != FR_FP64) return fail(c, FR_EUNSUPPORTED, "the adjoint is available for FP64 contexts");
  try {
    rk4_step_stash(c, u, dt_dev, stash, (hipStream_t)hip_stream);
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_rk_step_adjoint_stash(fr_ctx *c, double *stash, const double *dt_dev,
                                   const double *lam_np1, double *lam_n, void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!stash || !dt_dev || !lam_np1 || !lam_n) return fail(c, FR_EINVAL, "bad stash adjoint arguments");
  try {
    rk4_step_adjoint_stash(c, stash, dt_dev, lam_np1, lam_n, (hipStream_t)hip_stream);
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

// Captured segment graphs kept per context; the least recently used one
// makes room for a new argument set.
constexpr size_t kSegGraphs = 4;

fr_status fr_rk_segment_adjoint(fr_ctx *c, const double *u_seg0, const double *dt_dev,
                                int32_t nsteps, const double *lam_end, double *lam_seg0,
                                double *stash, void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u_seg0 || !dt_dev || !lam_end || !lam_seg0 || (nsteps > 0 && !stash) || nsteps < 0)
    return fail(c, FR_EINVAL, "bad segment adjoint arguments");
  if (c->prec != FR_FP64) return fail(c, FR_EUNSUPPORTED, "the adjoint is available for FP64 contexts");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    if (nsteps == 0) {
      rk4_segment_adjoint(c, u_seg0, dt_dev, 0, lam_end, lam_seg0, stash, s);
      return FR_OK;
    }
    // everything that allocates, uploads or synchronises happens before
    // the capture: adjoint operators, their tuning, the replay state
    ensure_adjoint(c, s);
    if (!c->adj_tuned) {
      c->adj_tuned = true;
      tune_adjoint_ops(c, s);
    }
    if (!c->d_seg_u) c->d_seg_u = dev_alloc<double>(c, c->total_len);
    fr_ctx::SegGraph *hit = nullptr;
    for (auto &g : c->seg_graphs)
      if (g.u0 == u_seg0 && g.dt == dt_dev && g.lam_end == lam_end && g.lam0 == lam_seg0 &&
          g.stash == stash && g.nsteps == nsteps)
        hit = &g;
    if (!hit) {
      if (c->seg_graphs.size() >= kSegGraphs) {
        auto old = std::min_element(c->seg_graphs.begin(), c->seg_graphs.end(),
                                    [](const fr_ctx::SegGraph &a, const fr_ctx::SegGraph &b) {
                                      return a.used < b.used;
                                    });
        release_graph_pair(old->graph, old->exec);
        c->seg_graphs.erase(old);
      }
      fr_ctx::SegGraph g{u_seg0, dt_dev, lam_end, lam_seg0, stash, nsteps, nullptr, nullptr, 0};
      capture(c, g.graph, g.exec, [&](hipStream_t cs) {
        rk4_segment_adjoint(c, u_seg0, dt_dev, nsteps, lam_end, lam_seg0, stash, cs);
      });
      c->seg_graphs.push_back(g);
      hit = &c->seg_graphs.back();
    }
    hit->used = ++c->seg_clock;
    hip_check(hipGraphLaunch(hit->exec, s), "graph launch");
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_integrate(fr_ctx *c, const double *u, int32_t kind, double *out, void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !out || kind != 0) return fail(c, FR_EINVAL, "bad integrate arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    for (auto &b : c->blocks)
      hip_check(fr::launch_elem_integrals(c->NV, c->D, b.Nu, b.ld, b.nelem, c->nchunk,
                                          c->nelem_total, b.d_wdjac, u + b.uoff,
                                          c->d_part + b.part_off, s),
                "elem integrals");
    hip_check(fr::launch_problem_sums(c->NV + 1, c->nproblems, c->nchunk, c->nelem_total,
                                      c->nslice, c->slice_len, c->d_pstart, c->d_plist, c->d_part,
                                      c->d_part2,
                                      out, s),
              "problem sums");
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_debug_multi(fr_ctx *c, int32_t step, int32_t mode, int32_t *state,
                         void *hip_stream) {
  if (!c || (step != 1 && step != 5 && step != 6 && step != 8)) return FR_EINVAL;
  if (step == 5 && !c->ns) return fail(c, FR_EINVAL, "no such step");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    if (mode > 0 && !kMultiBlockLaunches)
      return fail(c, FR_EUNSUPPORTED, "multi-block launches are switched off");
    if (mode >= 0) {
      // captured graphs hold the current slot tables as kernel arguments:
      // release them before the tables are freed and rebuilt
      hip_check(hipDeviceSynchronize(), "sync");
      release_graph(c);
      release_stepper_graphs(c);
      if (step == 6) {
        c->tflux_multi.on = false;
        if (mode > 0) build_tflux_multi(c, s);
      } else {
        free_multi(c->multi[step][0]);
        free_multi(c->multi[step][1]);
        if (mode > 0 && c->prec != FR_BF16X3) {
          build_multi_sparse(c, step, mode == 1 ? 1 : c->NV, s);
          build_multi_mfma(c, step, mode == 1 ? 1 : 2, s);
        }
      }
    }
    if (state) {
      *state = step == 6 ? (c->tflux_multi.on ? 4 : 0)
                         : (c->multi[step][0].on ? 1 : 0) | (c->multi[step][1].on ? 2 : 0);
    }
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_integrate_noalloc(fr_ctx *c, const double *u, int32_t kind, double *out,
                               void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !out || kind != 0) return fail(c, FR_EINVAL, "bad integrate arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  // element partials, then (several slices per problem) the slice partials,
  // 256-byte aligned
  const int64_t npart = (int64_t)c->nchunk * c->nelem_total * (c->NV + 1);
  const int64_t off2 = (npart + 31) / 32 * 32;
  const int64_t npart2 = c->nslice > 1 ? (int64_t)c->nproblems * c->nslice * (c->NV + 1) : 0;
  if (off2 + npart2 > fr::kIntegralScratchDoubles)
    return fail(c, FR_EINVAL,
                "fr_integrate_noalloc: this mesh needs " + std::to_string(off2 + npart2) +
                    " doubles of scratch; the fixed scratch holds " +
                    std::to_string(fr::kIntegralScratchDoubles) + " (use fr_integrate)");
  try {
    double *scr = nullptr;
    hip_check(fr::integral_scratch(&scr), "integral scratch address");
    // every partial the sums read is written first: nothing to clear
    for (auto &b : c->blocks)
      hip_check(fr::launch_elem_integrals(c->NV, c->D, b.Nu, b.ld, b.nelem, c->nchunk,
                                          c->nelem_total, b.d_wdjac, u + b.uoff,
                                          scr + b.part_off, s),
                "elem integrals");
    hip_check(fr::launch_problem_sums(c->NV + 1, c->nproblems, c->nchunk, c->nelem_total,
                                      c->nslice, c->slice_len, c->d_pstart, c->d_plist, scr,
                                      npart2 ? scr + off2 : nullptr, out, s),
              "problem sums");
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_reference_operator(int32_t etype, int32_t order, int32_t correction, int32_t which,
                                double *out, int64_t cap, int32_t *rows, int32_t *cols) {
  try {
    fr::RefOps R = fr::build_ref(etype, order, correction);
    const int D = R.ndims, Nu = R.nupts, Nf = R.nfpts;
    const std::vector<double> *v = nullptr;
    int r = 0, cc = 0;
    switch (which) {
      case 0: v = &R.M0; r = Nf; cc = Nu; break;
      case 1: v = &R.M3; r = Nu; cc = Nf; break;
      case 2: v = &R.M4p; r = D * Nu; cc = Nu; break;
      case 3: v = &R.M6; r = D * Nu; cc = Nf; break;
      case 4: v = &R.M1p; r = Nu; cc = D * Nu; break;
      case 5: v = &R.upts; r = Nu; cc = D; break;
      case 6: v = &R.fpts; r = Nf; cc = D; break;
      case 7: v = &R.fnorm; r = Nf; cc = D; break;
      case 8: v = &R.W; r = Nu; cc = 1; break;
      case 9: v = &R.fweight; r = Nf; cc = 1; break;
      case 10: v = &R.M4; r = D * Nu; cc = Nu; break;
      case 11: v = &R.M1; r = Nu; cc = D * Nu; break;
      default: return fail(nullptr, FR_EINVAL, "bad operator id");
    }
    if (rows) *rows = r;
    if (cols) *cols = cc;
    if (!out) return FR_OK;
    if (cap < (int64_t)v->size()) return fail(nullptr, FR_EINVAL, "output too small");
    std::memcpy(out, v->data(), v->size() * sizeof(double));
  } catch (const fr::SetupError &e) {
    return fail(nullptr, (fr_status)e.status, e.what());
  }
  return FR_OK;
}

fr_status fr_check_mesh(const fr_config *cfg, int32_t nblocks, const fr_block *blocks,
                        int64_t npairs, const fr_facepair *pairs, int64_t *npoint_pairs) {
  if (!cfg || !blocks || nblocks < 1 || npairs < 0 || (npairs > 0 && !pairs))
    return fail(nullptr, FR_EINVAL, "bad arguments");
  const int D = cfg->ndims;
  if (D != 2 && D != 3) return fail(nullptr, FR_EINVAL, "ndims must be 2 or 3");
  try {
    std::vector<fr::RefOps> refs;
    std::map<std::tuple<int, int, int>, int> refmap;
    std::vector<fr::BlockGeom> geoms;
    std::vector<int> block_ref;
    for (int bi = 0; bi < nblocks; ++bi) {
      const fr_block &B = blocks[bi];
      if (B.nelem < 1 || !B.nodes) return fail(nullptr, FR_EINVAL, "block without elements");
      if (block_too_large(B, D + 2)) return fail(nullptr, FR_EINVAL, kBlockTooLarge);
      if ((B.etype == FR_HEX) != (D == 3) || B.etype < 0 || B.etype > 2)
        return fail(nullptr, FR_EINVAL, "element type does not match ndims");
      auto key = std::make_tuple(B.etype, B.order, B.correction);
      if (!refmap.count(key)) {
        refmap[key] = (int)refs.size();
        refs.push_back(fr::build_ref(B.etype, B.order, B.correction));
      }
      block_ref.push_back(refmap[key]);
      geoms.push_back(fr::build_geom(refs[refmap[key]], B.geom_order, B.nelem, B.nodes,
                                     round_up(B.nelem, 16)));
    }
    std::vector<fr::FacePairIn> pin(npairs);
    for (int64_t k = 0; k < npairs; ++k) {
      const fr_facepair &P = pairs[k];
      pin[k] = fr::FacePairIn{P.lblock, P.lface, P.lelem, P.rblock, P.rface, P.relem,
                              {P.shift[0], P.shift[1], P.shift[2]}};
    }
    fr::PairTable T = fr::build_pairs(refs, geoms, block_ref, D, D + 2, pin.data(), npairs,
                                      nullptr, 0, 0, nullptr);
    if (npoint_pairs) *npoint_pairs = T.n;
  } catch (const fr::SetupError &e) {
    return fail(nullptr, (fr_status)e.status, e.what());
  } catch (const std::exception &e) {
    return fail(nullptr, FR_ENOMEM, e.what());
  }
  return FR_OK;
}

fr_status fr_debug_stage(fr_ctx *c, const double *u, int32_t stage, double *out,
                         void *hip_stream) {
  if (!c || !u || !out || stage < 1 || stage > 7) return FR_EINVAL;
  if (c->prec != FR_FP64) return fail(c, FR_EUNSUPPORTED, "debug stages are FP64 only");
  if (!c->ns && stage >= 2 && stage <= 5) return fail(c, FR_EINVAL, "no such stage for Euler");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    // Q~ itself exists only when step 4 runs on its own
    c->no_fuse = stage == 3;
    rhs_chain(c, u, nullptr, fr::EPI_NEGDIV, nullptr, nullptr, s, stage);
    c->no_fuse = false;
    const void *src = nullptr;
    int64_t n = 0;
    if (stage == 1 || stage == 7) { src = c->d_uf; n = c->uf_len; }
    else if (stage == 2) { src = c->d_qf; n = c->qf_len; }
    else if (stage == 5) { src = c->d_qf; n = c->qf_len; }
    else if (stage == 6) { src = c->cur.fto; n = c->ft_len; }
    else { src = c->d_ft; n = c->ft_len; }
    hip_check(hipMemcpyAsync(out, src, n * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
  } catch (const Fail &f) {
    c->no_fuse = false;
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_bench_step(fr_ctx *c, const double *u, int32_t step, int32_t nrep,
                        void *hip_stream) {
  if (!c || !u || step < 1 || step > 9 || nrep < 0) return FR_EINVAL;
  if (!c->ns && step >= 2 && step <= 5) return fail(c, FR_EINVAL, "no such step for Euler");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    rhs_chain(c, u, nullptr, fr::EPI_NEGDIV, nullptr, nullptr, s,
              step_before(c, std::min(step, 8)));
    // step 7 works in place, so its repeats read the previous repeat's
    // output: the same arithmetic and traffic on other values (timing only)
    if (step == 9) {
      // step 8 with the RK4 update of a middle stage, as the step graph runs
      // it (reads u and acc, writes acc and the next stage; dt = 0)
      fr::RkCoef rk;
      rk.a_next = 0.5; rk.b = 1.0 / 3; rk.first = 0; rk.last = 0;
      for (int i = 0; i < nrep; ++i)
        run_step(c, 8, c->d_stage, c->d_acc, fr::EPI_RK, &rk, c->d_tune_dt, s);
    }
    for (int i = 0; step <= 8 && i < nrep; ++i)
      run_step(c, step, u, c->d_acc, fr::EPI_NEGDIV, nullptr, nullptr, s);
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_debug_scratch_len(const fr_ctx *c, int32_t stage, int64_t *len) {
  if (!c || !len) return FR_EINVAL;
  *len = (stage == 1 || stage == 7) ? c->uf_len : ((stage == 2 || stage == 5) ? c->qf_len : c->ft_len);
  return FR_OK;
}

fr_status fr_debug_gemm(int32_t prec, int32_t M, int32_t K1, int32_t K2, const double *A,
                        const void *B1, const void *B2, int64_t ldb, void *C, int64_t N,
                        int32_t mbw, int32_t nc, int32_t wm, void *hip_stream) {
  if (!A || !B1 || !C || M < 1 || K1 < 1 || K2 < 0 || N < 16 || N % 16 || (K2 && !B2) ||
      ldb < N)
    return fail(nullptr, FR_EINVAL, "bad gemm arguments");
  if (prec != FR_FP64 && prec != FR_FP32 && prec != FR_BF16X3)
    return fail(nullptr, FR_EUNSUPPORTED, "precision");
  hipStream_t s = (hipStream_t)hip_stream;
  fr_ctx tmp;
  tmp.prec = prec;
  try {
    GemmOp op;
    std::vector<double> Av(A, A + (size_t)M * (K1 + K2));
    fr::GemmPlan p{mbw, nc, wm};
    if (mbw > 0 && (!fr::gemm_plan_valid(mbw, nc, wm, prec == FR_FP64 ? fr::PREC_F64
                                                       : (prec == FR_FP32 ? fr::PREC_F32
                                                                          : fr::PREC_BF16X3)) ||
                    wm < 1 || mbw * wm * 16 < M))
      throw Fail{FR_EINVAL, "bad plan"};
    if (mbw == 0 && (nc < 0 || wm != 0)) throw Fail{FR_EINVAL, "bad plan"};
    make_op(&tmp, op, Av, M, K1, K2, N, s, (mbw > 0 || nc > 0) ? &p : nullptr);
    if (mbw == 0 && nc > 0 && op.MBW != 0) throw Fail{FR_EINVAL, "operator is not sparse"};
    fr::GemmArgs g = gemm_args(op);
    g.B1 = B1; g.ldb1 = ldb; g.b1_f32 = 0;
    g.B2 = B2; g.ldb2 = ldb; g.b2_f32 = 0;
    g.C = C; g.ldc = N; g.c_f32 = prec != FR_FP64;
    g.N = N;
    hip_check(launch_op(op, prec == FR_FP64 ? fr::PREC_F64
                                : (prec == FR_FP32 ? fr::PREC_F32 : fr::PREC_BF16X3),
                        fr::EPI_STORE, g, 1, s),
              "gemm");
    hip_check(hipStreamSynchronize(s), "sync");
  } catch (const Fail &f) {
    for (void *p : tmp.allocs) hipFree(p);
    return fail(nullptr, f.st, f.msg);
  }
  for (void *p : tmp.allocs) hipFree(p);
  return FR_OK;
}

fr_status fr_measure_ceiling(int32_t kind, double *value, void *hip_stream) {
  if (!value || kind < 0 || kind > 2) return fail(nullptr, FR_EINVAL, "bad ceiling kind");
  hipError_t e = fr::measure_ceiling(kind, value, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(nullptr, FR_EDEVICE, hipGetErrorString(e));
  return FR_OK;
}

fr_status fr_bench_gemm(int32_t prec, int32_t M, int32_t K1, int32_t K2, int64_t N,
                        int32_t mbw, int32_t nc, int32_t wm, int32_t batch, int32_t nrep,
                        float *ms_per_launch, void *hip_stream) {
  if (!ms_per_launch || M < 1 || K1 < 1 || K2 < 0 || N < 16 || N % 16 || nrep < 1 || batch < 1)
    return fail(nullptr, FR_EINVAL, "bad gemm benchmark arguments");
  if (prec != FR_FP64 && prec != FR_FP32 && prec != FR_BF16X3)
    return fail(nullptr, FR_EUNSUPPORTED, "precision");
  hipStream_t s = (hipStream_t)hip_stream;
  fr_ctx tmp;
  tmp.prec = prec;
  const size_t es = prec == FR_FP64 ? 8 : 4;
  try {
    GemmOp op;
    std::vector<double> A((size_t)M * (K1 + K2), 0.5);
    fr::GemmPlan p{mbw, nc, wm};
    if (mbw > 0 && (!fr::gemm_plan_valid(mbw, nc, wm, prec == FR_FP64 ? fr::PREC_F64
                                                       : (prec == FR_FP32 ? fr::PREC_F32
                                                                          : fr::PREC_BF16X3)) ||
                    wm < 1 || mbw * wm * 16 < M))
      throw Fail{FR_EINVAL, "bad plan"};
    make_op(&tmp, op, A, M, K1, K2, N, s, mbw > 0 ? &p : nullptr);
    void *B1 = dev_alloc<char>(&tmp, (size_t)K1 * N * batch * es);
    void *B2 = dev_alloc<char>(&tmp, (size_t)(K2 ? K2 : 1) * N * es);
    void *C = dev_alloc<char>(&tmp, (size_t)M * N * batch * es);
    fr::GemmArgs g = gemm_args(op);
    g.B1 = B1; g.ldb1 = N; g.b1_f32 = prec != FR_FP64;
    g.B2 = B2; g.ldb2 = N; g.b2_f32 = prec != FR_FP64;
    g.C = C; g.ldc = N; g.c_f32 = prec != FR_FP64;
    g.N = N; g.sB1 = (int64_t)K1 * N; g.sC = (int64_t)M * N;
    const int gp = prec == FR_FP64 ? fr::PREC_F64 : (prec == FR_FP32 ? fr::PREC_F32 : fr::PREC_BF16X3);
    for (int w = 0; w < 3; ++w) hip_check(fr::launch_gemm(gp, fr::EPI_STORE, g, batch, s), "gemm");
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    hip_check(hipEventRecord(e0, s), "record");
    for (int w = 0; w < nrep; ++w) hip_check(fr::launch_gemm(gp, fr::EPI_STORE, g, batch, s), "gemm");
    hip_check(hipEventRecord(e1, s), "record");
    hip_check(hipEventSynchronize(e1), "sync");
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    *ms_per_launch = ms / nrep;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  } catch (const Fail &f) {
    hipDeviceSynchronize();
    for (void *q : tmp.allocs) hipFree(q);
    tmp.allocs.clear();
    return fail(nullptr, f.st, f.msg);
  }
  hipDeviceSynchronize();
  for (void *q : tmp.allocs) hipFree(q);
  tmp.allocs.clear();
  return FR_OK;
}

fr_status fr_get_gemm_plan(const fr_ctx *c, int32_t block, int32_t step, int32_t *mbw,
                           int32_t *nc, int32_t *wm) {
  if (!c || block < 0 || block >= (int)c->blocks.size() || !mbw || !nc || !wm) return FR_EINVAL;
  const BlockRT &b = c->blocks[block];
  const GemmOp *op = step == 1 ? &b.m0 : step == 3 ? &b.s3 : step == 5 ? &b.m5 : step == 8 ? &b.s8 : nullptr;
  if (!op || (!c->ns && (step == 3 || step == 5))) return FR_EINVAL;
  *mbw = op->MBW; *nc = op->NC; *wm = op->WM;
  return FR_OK;
}

fr_status fr_debug_set_plan(fr_ctx *c, int32_t block, int32_t step, int32_t mbw, int32_t nc,
                            int32_t wm, void *hip_stream) {
  if (!c || block < 0 || block >= (int)c->blocks.size()) return FR_EINVAL;
  BlockRT &b = c->blocks[block];
  hipStream_t s = (hipStream_t)hip_stream;
  if (step == 13 || step == 14) {
    // M0^T, or (M1 - M3 M2)^T, of the adjoint (set up and tuned first, so
    // the plan sticks)
    if (c->prec != FR_FP64) return fail(c, FR_EUNSUPPORTED, "the adjoint is FP64 only");
    try {
      ensure_adjoint(c, s);
      if (!c->adj_tuned) {
        c->adj_tuned = true;
        tune_adjoint_ops(c, s);
      }
    } catch (const Fail &f) {
      return fail(c, f.st, f.msg);
    }
  }
  GemmOp *op = step == 1 ? &b.m0 : step == 3 ? &b.s3 : step == 5 ? &b.m5 : step == 8 ? &b.s8
               : step == 13 ? &b.t_m0 : step == 14 ? &b.t_m1 : nullptr;
  if (!op || (!c->ns && (step == 3 || step == 5))) return fail(c, FR_EINVAL, "no such step");
  // a forced plan runs as it is: no multi-block launch of this step.  Graphs
  // captured before hold the old plan's kernel arguments (operator copies,
  // slot tables): release them before anything they point at is freed.
  hipDeviceSynchronize();
  release_graph(c);
  release_stepper_graphs(c);
  if (step == 1 || step == 5 || step == 8) {
    free_multi(c->multi[step][0]);
    free_multi(c->multi[step][1]);
  }
  try {
    fr::GemmPlan p{mbw, nc, wm};
    if (mbw > 0) {
      const int gp = c->prec == FR_FP64 ? fr::PREC_F64
                     : (c->prec == FR_FP32 ? fr::PREC_F32 : fr::PREC_BF16X3);
      if (!fr::gemm_plan_valid(mbw, nc, wm, gp) || wm < 1 || mbw * wm * 16 < op->M)
        throw Fail{FR_EINVAL, "bad matrix-core plan"};
      op->d_A = pack_upload(c, *op, p, s, true);
    } else {
      if (!op->sp.colidx) throw Fail{FR_EINVAL, "operator has no sparse-row form"};
      const bool staged = wm & kPlanStaged, fused = wm & kPlanFusedGradT;
      const bool fflux = wm & kPlanFusedFlux, fvjp = wm & kPlanFusedFluxVjp;
      if (nc < 1 || wm < 0 || wm > 31 || (fused && step != 3) ||
          (fvjp && (step != 14 || wm != (kPlanFields | kPlanFusedFluxVjp) ||
                    op->sp.width > FR_SPOP_GRADT_FIELDS_WMAX)) ||
          (fflux && (wm & ~kPlanStaged) != kPlanFusedAll) || (fflux && staged) ||
          (fflux && op->sp.width > FR_SPOP_GRADT_FIELDS_WMAX) ||
          (staged && ((wm & kPlanFields) || !staged_ok(*op, fused, c->D))) ||
          (wm == (kPlanFusedGradT | kPlanFields) && op->sp.width > FR_SPOP_GRADT_FIELDS_WMAX) ||
          (step == 13 && c->ns && (wm & kPlanFields) && op->sp.width > FR_SPOP_GRADT_FIELDS_WMAX))
        throw Fail{FR_EINVAL, "bad sparse-row plan"};
      op->d_A = nullptr;
      apply_sparse_plan(*op, p, c->NV);
    }
    op->MBW = mbw; op->NC = nc; op->WM = wm;
    hip_check(hipStreamSynchronize(s), "sync");
    // captured steps hold the previous plan's launches
    release_graph(c);
    release_stepper_graphs(c);
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

fr_status fr_integrate_grad(fr_ctx *c, const double *u, int32_t kind, double *grad,
                            void *hip_stream) {
  if (!c) return FR_EINVAL;
  if (!u || !grad || kind != 1) return fail(c, FR_EINVAL, "bad integrate_grad arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    for (auto &b : c->blocks)
      hip_check(fr::launch_ke_grad(c->NV, c->D, b.Nu, b.ld, b.nelem, b.d_wdjac, u + b.uoff,
                                   grad + b.uoff, s), "ke grad");
  } catch (const Fail &f) {
    return fail(c, f.st, f.msg);
  }
  return FR_OK;
}

const char *fr_last_error(const fr_ctx *c) {
  return c ? c->err.c_str() : g_setup_error.c_str();
}

void fr_destroy(fr_ctx *c) {
  if (!c) return;
  hipDeviceSynchronize();
  release_graph(c);
  release_stepper_graphs(c);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  for (auto &row : c->multi)
    for (auto &ml : row) free_multi(ml);
  for (void *p : c->allocs) hipFree(p);
  delete c;
}

}  // extern "C"
