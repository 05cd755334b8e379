// Sparse-row application of an operator matrix: C = A [B1; B2] where A has
// few non-zeros per row (kernel template; instantiated in spop.hip for one
// field per thread and in spop_fields.hip for all fields per thread).
//
// With Gauss-Legendre points on quads and hexes every Appendix A operator
// couples only points on one coordinate line (interpolation to a face,
// differentiation along a line, the DG lifting along the face normal), so a
// row holds O(p) non-zeros out of up to a few hundred.  Applying such an
// operator as a dense product would make an HBM-bound step compute-bound.
//
// Threads of a wavefront take consecutive elements (coalesced).  With F = 1
// a thread owns one state column (field, element); with F = N_V it owns an
// element and produces every field of it, so the operator entries (scalar
// loads), the per-point metric terms of the epilogues and the step size are
// fetched once for all fields, and each row issues F x W independent loads.
// Each workgroup row takes `rpg` operator rows.  The operator is stored
// padded to a fixed width W per row (ELL: padding entries have value 0 and
// repeat a real column), W is a template parameter, so all loads of a row
// are issued back to back; column indices and values are wave-uniform.
// The grid is one-dimensional and XCD-aware: workgroups are dealt
// round-robin to the 8 XCDs, and the linear id is remapped so that each XCD
// runs all row groups of one column tile back to back; re-reads of that
// tile's B rows then hit the XCD's L2 while they are still there.
#pragma once

#include "buffer.h"
#include "kernels.h"
#include "physics.h"

namespace fr {

// OFF: every entry's B row comes from the precomputed byte offsets g.roff
// (one buffer resource over both panels, the row offset as the instruction's
// scalar offset): no scalar address arithmetic per entry.
// MULTI (with OFF): a multi-block launch that reads each workgroup's block
// from g.slots.  A separate instantiation: the slot table is read through a
// generic pointer, whose loads the compiler takes as divergent, and in a
// shared kernel that would turn every gather of the single-block launch into
// a waterfall loop over lanes.
template <typename T, int EPI, int W, typename TB1, typename TB2, typename TC, int DG, int F,
          bool OFF = false, bool MULTI = false>
__global__ __launch_bounds__(256) void spop_kernel(GemmArgs g,
                                                   const int32_t *__restrict__ colidx,
                                                   const double *__restrict__ vals, int rpg,
                                                   int ngroups) {
  static_assert(!OFF || (EPI != EPI_ADDT && EPI != EPI_TFVJP && EPI != EPI_GRADT &&
                         EPI != EPI_GRADTF),
                "precomputed gathers and multi-block launches: store, add, -1/J, RK only");
  static_assert(!MULTI || OFF, "multi-block launches use the precomputed gathers");
  // multi-block launch (precomputed-gather variant): this workgroup's
  // block, its operator and its index within the block
  int64_t L = blockIdx.x;
  if constexpr (MULTI) {
    const LaunchSlot *sl = nullptr;
    L = take_slot(g, L, sizeof(TB1), sizeof(TB2), sizeof(TC), &sl);
    vals = sl->vals;
    rpg = sl->rpg;
    ngroups = sl->ngroups;
  }
  // linear id L -> XCD L % 8; the j-th workgroup of an XCD takes row group
  // j % ngroups of column tile 8 (j / ngroups) + L % 8 (tiles padded to a
  // multiple of 8 by the launch, and every block's range of a multi-block
  // launch starts at a multiple of 8)
  const int64_t j = L >> 3;
  const int64_t tile = (j / ngroups) * 8 + (L & 7);
  const int rgrp = (int)(j % ngroups);
  // F == 1: t is the state column alpha * ld + n; F > 1: t is the element n
  const int64_t t = tile * 256 + threadIdx.x;
  if (t >= (F == 1 ? g.N : g.ld)) return;
  const int r0 = rgrp * rpg;
  constexpr bool GT = EPI == EPI_GRADT || EPI == EPI_GRADTF || EPI == EPI_TFVJP;
  const int rmax = GT ? g.Nu : g.M;  // EPI_ADDT: M = Nu
  const int r1 = r0 + rpg < rmax ? r0 + rpg : rmax;
  const TB1 *__restrict__ B1b = (const TB1 *)g.B1 + (int64_t)blockIdx.y * g.sB1;
  const TB1 *__restrict__ B1 = B1b + t;
  const TB2 *__restrict__ B2 = (const TB2 *)g.B2 + t;
  int64_t n = 0;
  if (EPI == EPI_NEGDIV || EPI == EPI_RK || GT || EPI == EPI_ADDT || EPI == EPI_RKADJ)
    n = F == 1 ? t % g.ld : t;
  const bool live = n < g.nelem;
  double dtv = 0;
  if ((EPI == EPI_RK || EPI == EPI_RKADJ) && live) dtv = g.dt[g.prob ? g.prob[n] : 0];
  const int K1 = g.K1;
  // both panels have the row stride ldb, and N <= ldb < 2^29 (checked by
  // the launcher): a row of B spans under 4 GiB
  const int32_t ldb = (int32_t)g.ldb1;
  const int64_t fs = F == 1 ? 0 : g.ld;
  // row k of the stacked operand [B1; B2] starts k ldb values after the
  // base of its panel, so the panel of an entry costs one uniform select,
  // not a branch and a second product
  const uint32_t rsb = (uint32_t)ldb * (uint32_t)sizeof(TB1);  // row stride, bytes
  // where row 0 of [B1; B2] would start if B2 were panel 1 (row K1 is B2's row 0)
  // (integer arithmetic: B2 is null for single-panel operators, never read)
  const char *const b2row0 = (const char *)((uintptr_t)g.B2 - (uint64_t)K1 * rsb);
  // byte offset of field a's column within a row of B
  uint32_t toff[F];
#pragma unroll
  for (int a = 0; a < F; ++a) toff[a] = (uint32_t)((t + a * fs) * (int64_t)sizeof(TB1));

  // OFF: one resource from rbase (this workgroup's batch slice)
  const __amdgpu_buffer_rsrc_t rsoff = __builtin_amdgcn_make_buffer_rsrc(
      OFF ? (void *)((const char *)g.rbase + (int64_t)blockIdx.y * g.sB1 * (int64_t)sizeof(TB1))
          : nullptr,
      0, -1, kRawBufferWord3);

  // acc[a] = row `row` of A times field a's column (of panel 1 shifted by
  // boff elements: a batch slice)
  auto row_product = [&](int row, T(&acc)[F], int64_t boff = 0) {
    const double *__restrict__ cv = vals + (int64_t)row * W;
    if constexpr (OFF) {
      static_assert(sizeof(TB1) == sizeof(TB2), "one resource spans both panels");
      const uint32_t *__restrict__ ro = g.roff + (int64_t)row * W;
      uint32_t ko[W];
#pragma unroll
      for (int e = 0; e < W; ++e) ko[e] = ro[e];
      T b[F][W];
#pragma unroll
      for (int e = 0; e < W; ++e)
#pragma unroll
        for (int a = 0; a < F; ++a) b[a][e] = (T)load_row<TB1>(rsoff, toff[a], ko[e]);
#pragma unroll
      for (int a = 0; a < F; ++a) {
        T s = 0;
#pragma unroll
        for (int e = 0; e < W; ++e) s += (T)cv[e] * b[a][e];
        acc[a] = s;
      }
      return;
    }
    const int32_t *__restrict__ ci = colidx + (int64_t)row * W;
    int32_t kc[W];
#pragma unroll
    for (int e = 0; e < W; ++e) kc[e] = ci[e];
    // row 0 of [B1; B2] as seen from each panel (panel 1 shifted by boff);
    // base2 is formed from B2's own pointer so that the compiler keeps the two
    // bases apart and picks one with a single 64-bit select
    const char *base1 = (const char *)B1b + boff * (int64_t)sizeof(TB1);
    const char *base2 = b2row0;
    T b[F][W];
#pragma unroll
    for (int e = 0; e < W; ++e) {
      const int k = kc[e];
      if constexpr (sizeof(TB1) == sizeof(TB2)) {
        const char *rowp = (k < K1 ? base1 : base2) + (uint64_t)(uint32_t)k * rsb;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)rowp, 0, -1, kRawBufferWord3);
#pragma unroll
        for (int a = 0; a < F; ++a) b[a][e] = (T)load_row<TB1>(rs, toff[a]);
      } else {
#pragma unroll
        for (int a = 0; a < F; ++a)
          b[a][e] = k < K1 ? (T)B1[(int64_t)k * ldb + a * fs]
                           : (T)B2[(int64_t)(k - K1) * ldb + a * fs];
      }
    }
#pragma unroll
    for (int a = 0; a < F; ++a) {
      T s = 0;
#pragma unroll
      for (int e = 0; e < W; ++e) s += (T)cv[e] * b[a][e];
      acc[a] = s;
    }
  };

  if constexpr (EPI == EPI_ADDT) {
    // row rho of batch slices d < DG (panel 1 only), added to C, then
    // qtb_i = (1/J) sum_j S_ij qb_j at the point
    const int64_t plane = (int64_t)g.Nu * g.ld;
    double *C = (double *)g.C;
    for (int rho = r0; rho < r1; ++rho) {
      T pr[DG][F];
#pragma unroll
      for (int d = 0; d < DG; ++d) row_product(rho, pr[d], d * g.sB1);
      double qb[DG][F];
#pragma unroll
      for (int d = 0; d < DG; ++d)
#pragma unroll
        for (int a = 0; a < F; ++a)
          qb[d][a] = C[d * g.sC + (int64_t)rho * g.ldc + t + a * fs] + (double)pr[d][a];
      const int64_t pt = (int64_t)rho * g.ld + n;
      if (live) {
        const double rj = g.rcpdjac[pt];
        double S[DG][DG];
#pragma unroll
        for (int i = 0; i < DG; ++i)
#pragma unroll
          for (int jj = 0; jj < DG; ++jj) S[i][jj] = g.smat[(i * DG + jj) * plane + pt];
#pragma unroll
        for (int a = 0; a < F; ++a)
#pragma unroll
          for (int i = 0; i < DG; ++i) {
            double si = 0;
#pragma unroll
            for (int jj = 0; jj < DG; ++jj) si += S[i][jj] * qb[jj][a];
            C[i * g.sC + (int64_t)rho * g.ldc + t + a * fs] = rj * si;
          }
      } else {
#pragma unroll
        for (int d = 0; d < DG; ++d)
#pragma unroll
          for (int a = 0; a < F; ++a) C[d * g.sC + (int64_t)rho * g.ldc + t + a * fs] = qb[d][a];
      }
    }
    return;
  }
  if constexpr (EPI == EPI_TFVJP) {
    // rows d Nu + rho, d < DG, of the points rho in [r0, r1): F~b of the point
    static_assert(F == DG + 2, "the flux needs every field of a point");
    const int64_t plane = (int64_t)g.Nu * g.ld;
    double *C = (double *)g.C;
    for (int rho = r0; rho < r1; ++rho) {
      T Fb[DG][F];
#pragma unroll
      for (int d = 0; d < DG; ++d) row_product(d * g.Nu + rho, Fb[d]);
      const int64_t pt = (int64_t)rho * g.ld + n;
      const int64_t up = (int64_t)rho * g.ldc + t;
      if (live) {
        double S[DG][DG];
#pragma unroll
        for (int i = 0; i < DG; ++i)
#pragma unroll
          for (int jj = 0; jj < DG; ++jj) S[i][jj] = g.smat[(i * DG + jj) * plane + pt];
        double u[F], fb[DG][F], ub[F];
#pragma unroll
        for (int a = 0; a < F; ++a) { u[a] = g.uprim[up + a * fs]; ub[a] = 0; }
#pragma unroll
        for (int jj = 0; jj < DG; ++jj)
#pragma unroll
          for (int a = 0; a < F; ++a) {
            double sj = 0;
#pragma unroll
            for (int i = 0; i < DG; ++i) sj += S[i][jj] * (double)Fb[i][a];
            fb[jj][a] = sj;
          }
        inviscid_flux_vjp<DG>(u, g.gamma, fb, 0.0, nullptr, ub);
        if (g.qprim) {
          double q[DG][F], qb[DG][F], nfb[DG][F];
#pragma unroll
          for (int jj = 0; jj < DG; ++jj)
#pragma unroll
            for (int a = 0; a < F; ++a) {
              q[jj][a] = g.qprim[(int64_t)(jj * g.Nu + rho) * g.ldc + t + a * fs];
              qb[jj][a] = 0;
              nfb[jj][a] = -fb[jj][a];
            }
          viscous_flux_vjp<DG>(u, q, g.gamma, g.mu, g.prandtl, nfb, ub, qb);
#pragma unroll
          for (int jj = 0; jj < DG; ++jj)
#pragma unroll
            for (int a = 0; a < F; ++a) C[(int64_t)(jj * g.Nu + rho) * g.ldc + t + a * fs] = qb[jj][a];
        }
#pragma unroll
        for (int a = 0; a < F; ++a) g.out[up + a * fs] = ub[a];
      } else {
#pragma unroll
        for (int a = 0; a < F; ++a) {
          g.out[up + a * fs] = 0.0;
          if (g.qprim)
#pragma unroll
            for (int jj = 0; jj < DG; ++jj) C[(int64_t)(jj * g.Nu + rho) * g.ldc + t + a * fs] = 0.0;
        }
      }
    }
    return;
  } else if constexpr (GT) {
    // rows d Nu + rho, d < DG, of the points rho in [r0, r1) (r1 <= Nu)
    static_assert(EPI != EPI_GRADTF || F == DG + 2, "the flux needs every field of a point");
    const int64_t plane = (int64_t)g.Nu * g.ld;
    TC *C = (TC *)g.C;
    for (int rho = r0; rho < r1; ++rho) {
      T qt[DG][F];
#pragma unroll
      for (int d = 0; d < DG; ++d) row_product(d * g.Nu + rho, qt[d]);
      const int64_t pt = (int64_t)rho * g.ld + n;
      if (live) {
        const double rj = g.rcpdjac[pt];
        double S[DG][DG];
#pragma unroll
        for (int i = 0; i < DG; ++i)
#pragma unroll
          for (int jj = 0; jj < DG; ++jj) S[i][jj] = g.smat[(i * DG + jj) * plane + pt];
        // Q of the point as stored (rounded to TC), kept for the flux
        double q[DG][F];
#pragma unroll
        for (int a = 0; a < F; ++a)
#pragma unroll
          for (int jj = 0; jj < DG; ++jj) {
            double sj = 0;
#pragma unroll
            for (int i = 0; i < DG; ++i) sj += S[i][jj] * (double)qt[i][a];
            const TC qv = (TC)(rj * sj);
            C[(int64_t)(jj * g.Nu + rho) * g.ldc + t + a * fs] = qv;
            q[jj][a] = (double)qv;
          }
        if constexpr (EPI == EPI_GRADTF) {
          // the FP64 state of the point (rows rho of every field)
          const double *__restrict__ up = g.uprim + (int64_t)rho * ldb + t;
          double u[F], f[DG][F], fv[DG][F], p, v[DG];
#pragma unroll
          for (int a = 0; a < F; ++a) u[a] = up[a * fs];
          inviscid_flux<DG>(u, g.gamma, f, p, v);
          viscous_flux<DG>(u, q, g.gamma, g.mu, g.prandtl, fv);
#pragma unroll
          for (int jj = 0; jj < DG; ++jj)
#pragma unroll
            for (int a = 0; a < F; ++a) f[jj][a] -= fv[jj][a];
          if (g.devflux) {
            // deviation form: less the inviscid flux of the element's
            // reference state (its first solution point)
            double ub[F], fb[DG][F], pb, vb[DG];
#pragma unroll
            for (int a = 0; a < F; ++a) ub[a] = g.uprim[t + a * fs];
            inviscid_flux<DG>(ub, g.gamma, fb, pb, vb);
#pragma unroll
            for (int jj = 0; jj < DG; ++jj)
#pragma unroll
              for (int a = 0; a < F; ++a) f[jj][a] -= fb[jj][a];
          }
          TC *Fo = (TC *)g.fout;
#pragma unroll
          for (int i = 0; i < DG; ++i)
#pragma unroll
            for (int a = 0; a < F; ++a) {
              double sf = 0;
#pragma unroll
              for (int jj = 0; jj < DG; ++jj) sf += S[i][jj] * f[jj][a];
              Fo[(int64_t)(i * g.Nu + rho) * g.ldc + t + a * fs] = (TC)sf;
            }
        }
      } else {
#pragma unroll
        for (int a = 0; a < F; ++a)
#pragma unroll
          for (int jj = 0; jj < DG; ++jj) {
            C[(int64_t)(jj * g.Nu + rho) * g.ldc + t + a * fs] = (TC)qt[jj][a];
            if constexpr (EPI == EPI_GRADTF)
              ((TC *)g.fout)[(int64_t)(jj * g.Nu + rho) * g.ldc + t + a * fs] = (TC)0;
          }
      }
    }
    return;
  }
  auto row_step = [&](int row) {
    // RK4 update: the state and register values of this row are loaded
    // before the gathers, so that their latency overlaps the product's
    // instead of following it (the state is read unless this is the last
    // stage, the register unless this is a first stage that is not also the
    // last one, as in forward Euler; buffer loads from this row of each
    // array, with an empty range where the stage does not read it: 0 comes back
    // with no memory access and no branch, so nothing waits before the
    // gathers are issued; readfirstlane keeps the uniform ranges in scalar
    // registers, which a buffer resource must be in)
    double u0v[F], accv[F];
    if constexpr (EPI == EPI_RK) {
      const __amdgpu_buffer_rsrc_t rso = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(g.out + (int64_t)row * g.ldc), 0,
          __builtin_amdgcn_readfirstlane(g.rk.last ? 0 : -1), kRawBufferWord3);
      const __amdgpu_buffer_rsrc_t rsa = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(g.acc + (int64_t)row * g.ldc), 0,
          __builtin_amdgcn_readfirstlane(g.rk.first && !g.rk.last ? 0 : -1), kRawBufferWord3);
#pragma unroll
      for (int a = 0; a < F; ++a) {
        // within one row of N < 2^29 columns: the byte offset fits 32 bits
        const uint32_t off = (uint32_t)((t + a * fs) * (int64_t)sizeof(double));
        u0v[a] = load_row<double>(rso, off);
        accv[a] = load_row<double>(rsa, off);
      }
    }
    T acc[F];
    row_product(row, acc);
    double rj = 0;
    if (EPI == EPI_NEGDIV || EPI == EPI_RK || EPI == EPI_RKADJ)
      rj = live ? g.rcpdjac[(int64_t)row * g.ld + n] : 0.0;
#pragma unroll
    for (int a = 0; a < F; ++a) {
      const int64_t idx = (int64_t)row * g.ldc + t + a * fs;
      if (EPI == EPI_STORE) {
        ((TC *)g.C)[(int64_t)blockIdx.y * g.sC + idx] = (TC)acc[a];
      } else if (EPI == EPI_ADD) {
        TC *cp = (TC *)g.C + (int64_t)blockIdx.y * g.sC + idx;
        *cp = (TC)((double)*cp + (double)acc[a]);
      } else if (EPI == EPI_RKADJ) {
        const double w = (double)((const TC *)g.C)[idx] + (double)acc[a];
        g.acc[idx] += w;
        if (!g.rk.last)
          g.out[idx] = live ? -rj * (g.rk.a_next * dtv * g.stage[idx] + g.rk.b * dtv * w) : 0.0;
      } else {
        // padding columns: exactly 0 whatever they hold (even NaN)
        const double kk = live ? -rj * (double)acc[a] : 0.0;
        if (EPI == EPI_NEGDIV) {
          g.out[idx] = kk;
        } else {
          const double bdt = g.rk.b * dtv * kk;
          if (g.rk.last) {
            g.out[idx] = accv[a] + bdt;
          } else {
            const double u0 = u0v[a];
            g.acc[idx] = (g.rk.first ? u0 : accv[a]) + bdt;
            g.stage[idx] = u0 + g.rk.a_next * dtv * kk;
          }
        }
      }
    }
  };
  if constexpr (EPI == EPI_RK) {
    // (readfirstlane is convergent: this loop is not unrolled)
#pragma unroll 1
    for (int row = r0; row < r1; ++row) row_step(row);
  } else {
#pragma unroll 2
    for (int row = r0; row < r1; ++row) row_step(row);
  }
}

// Column tiles of 256 threads, padded to a multiple of the 8 XCDs.
template <int F>
inline int64_t spop_tiles(const GemmArgs &g) {
  const int64_t threads = F == 1 ? g.N : g.ld;
  return ((threads + 255) / 256 + 7) / 8 * 8;
}

template <typename T, int EPI, int W, typename TB1, typename TB2, typename TC, int F>
void spop_go(const GemmArgs &g, const SparseOp &sp, dim3 grid, int ngroups, hipStream_t s) {
  // precomputed gathers where both panels have one element size (the
  // epilogues without point data: store, add, -1/J, RK update)
  constexpr bool off_ok = sizeof(TB1) == sizeof(TB2) && EPI != EPI_ADD && EPI != EPI_RKADJ;
  if (off_ok && g.roff)
    spop_kernel<T, EPI, W, TB1, TB2, TC, 0, F, off_ok><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
  else
    spop_kernel<T, EPI, W, TB1, TB2, TC, 0, F><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
}

// Multi-block launch (g.slots): the precomputed-gather kernel over g.nwg
// workgroups, each block's operator and row groups taken from its slot.
template <typename T, int EPI, int W, int F>
void spop_multi_w(const GemmArgs &g, int batch, hipStream_t s) {
  dim3 grid((unsigned)g.nwg, batch);
  if constexpr (sizeof(T) == 8) {
    spop_kernel<T, EPI, W, double, double, double, 0, F, true, true><<<grid, 256, 0, s>>>(g, nullptr, nullptr, 1, 1);
  } else if constexpr (EPI == EPI_NEGDIV || EPI == EPI_RK) {
    spop_kernel<T, EPI, W, float, float, double, 0, F, true, true><<<grid, 256, 0, s>>>(g, nullptr, nullptr, 1, 1);
  } else {
    if (!g.b1_f32)
      spop_kernel<T, EPI, W, double, double, float, 0, F, true, true><<<grid, 256, 0, s>>>(g, nullptr, nullptr, 1, 1);
    else
      spop_kernel<T, EPI, W, float, float, float, 0, F, true, true><<<grid, 256, 0, s>>>(g, nullptr, nullptr, 1, 1);
  }
}

template <int F>
hipError_t launch_spop_multi_f(int prec, int epi, const GemmArgs &g, int width, int batch,
                               hipStream_t s) {
  if (!g.slots || g.nslots < 1 || g.nwg < 1) return hipErrorInvalidValue;
  // the -1/J and RK4 epilogues write through out (and the RK registers)
  if ((epi == EPI_NEGDIV || epi == EPI_RK) && !g.out) return hipErrorInvalidValue;
  if (epi == EPI_RK && (!g.acc || !g.dt || (!g.rk.last && !g.stage))) return hipErrorInvalidValue;
  if (epi == EPI_STORE && !g.C) return hipErrorInvalidValue;
  if (prec == PREC_F32 && epi == EPI_STORE && g.b1_f32 && !g.b2_f32 && g.B2)
    return hipErrorInvalidValue;  // panels of two element sizes
#define FR_W(W_)                                                                     \
  case W_:                                                                           \
    if (prec == PREC_F64) {                                                          \
      if (epi == EPI_STORE) spop_multi_w<double, EPI_STORE, W_, F>(g, batch, s);     \
      else if (epi == EPI_NEGDIV) spop_multi_w<double, EPI_NEGDIV, W_, F>(g, batch, s); \
      else if (epi == EPI_RK) spop_multi_w<double, EPI_RK, W_, F>(g, batch, s);     \
      else return hipErrorInvalidValue;                                              \
    } else if (prec == PREC_F32) {                                                   \
      if (epi == EPI_STORE) spop_multi_w<float, EPI_STORE, W_, F>(g, batch, s);      \
      else if (epi == EPI_NEGDIV) spop_multi_w<float, EPI_NEGDIV, W_, F>(g, batch, s); \
      else if (epi == EPI_RK) spop_multi_w<float, EPI_RK, W_, F>(g, batch, s);      \
      else return hipErrorInvalidValue;                                              \
    } else {                                                                         \
      return hipErrorInvalidValue;                                                   \
    }                                                                                \
    break;
  switch (width) {
    FR_SPOP_WIDTHS(FR_W)
    default: return hipErrorInvalidValue;
  }
#undef FR_W
  return hipGetLastError();
}

template <typename T, int EPI, int W, int F>
void spop_launch_w(const GemmArgs &g, const SparseOp &sp, int batch, hipStream_t s) {
  const int ngroups = (g.M + sp.rpg - 1) / sp.rpg;
  dim3 grid((unsigned)(spop_tiles<F>(g) * ngroups), batch);
  if constexpr (sizeof(T) == 8) {
    spop_go<T, EPI, W, double, double, double, F>(g, sp, grid, ngroups, s);
  } else if constexpr (EPI == EPI_NEGDIV || EPI == EPI_RK) {
    spop_go<T, EPI, W, float, float, double, F>(g, sp, grid, ngroups, s);
  } else {
    if (!g.b1_f32)
      spop_go<T, EPI, W, double, double, float, F>(g, sp, grid, ngroups, s);
    else if (!g.b2_f32)
      spop_go<T, EPI, W, float, double, float, F>(g, sp, grid, ngroups, s);
    else
      spop_go<T, EPI, W, float, float, float, F>(g, sp, grid, ngroups, s);
  }
}

template <typename T, int EPI, int W, int DG, int F>
void spop_launch_gradt(const GemmArgs &g, const SparseOp &sp, hipStream_t s) {
  const int ngroups = (g.Nu + sp.rpg - 1) / sp.rpg;
  dim3 grid((unsigned)(spop_tiles<F>(g) * ngroups), 1);
  if constexpr (sizeof(T) == 8)
    spop_kernel<T, EPI, W, double, double, double, DG, F><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
  else  // FP32 contexts: C^f and the state's deviation (deviation form), both FP32
    spop_kernel<T, EPI, W, float, float, float, DG, F><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
}

template <int W, int DG, int F>
void spop_launch_addt(const GemmArgs &g, const SparseOp &sp, hipStream_t s) {
  const int ngroups = (g.M + sp.rpg - 1) / sp.rpg;
  dim3 grid((unsigned)(spop_tiles<F>(g) * ngroups), 1);
  spop_kernel<double, EPI_ADDT, W, double, double, double, DG, F><<<grid, 256, 0, s>>>(
      g, sp.colidx, sp.vals, sp.rpg, ngroups);
}

template <int F>
hipError_t spop_addt_t(const GemmArgs &g, const SparseOp &sp, hipStream_t s) {
  if ((g.D != 2 && g.D != 3) || g.Nu != g.M || g.K2 != 0 || !g.smat) return hipErrorInvalidValue;
  constexpr int DG = F == 4 ? 2 : 3;
  if (F > 1 && g.D != DG) return hipErrorInvalidValue;
  switch (sp.width) {
#define FR_W(W_)                                                          \
  case W_:                                                                \
    if constexpr (F > 1 && W_ > FR_SPOP_GRADT_FIELDS_WMAX)                \
      return hipErrorInvalidValue;                                        \
    else if constexpr (F > 1) spop_launch_addt<W_, DG, F>(g, sp, s);      \
    else if (g.D == 3) spop_launch_addt<W_, 3, F>(g, sp, s);              \
    else spop_launch_addt<W_, 2, F>(g, sp, s);                            \
    break;
    FR_SPOP_WIDTHS(FR_W)
#undef FR_W
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int F, int EPI = EPI_GRADT>
hipError_t spop_gradt_t(const GemmArgs &g, const SparseOp &sp, hipStream_t s) {
  if ((g.D != 2 && g.D != 3) || g.Nu * g.D != g.M || !g.smat) return hipErrorInvalidValue;
  if (sizeof(T) == 4 && (!g.b1_f32 || !g.b2_f32 || !g.c_f32)) return hipErrorInvalidValue;
  if (EPI == EPI_GRADTF && !g.uprim) return hipErrorInvalidValue;
  // all fields per thread: F is the field count D + 2
  constexpr int DG = F == 4 ? 2 : 3;
  if (F > 1 && g.D != DG) return hipErrorInvalidValue;
  if constexpr (EPI == EPI_GRADTF) {
    if (F == 1 || !g.fout || g.fout == g.C) return hipErrorInvalidValue;
  }
  if constexpr (EPI == EPI_TFVJP) {
    if (F == 1 || sizeof(T) != 8 || !g.uprim || !g.out || g.K2 != 0 || g.K1 != g.Nu)
      return hipErrorInvalidValue;
  }
  switch (sp.width) {
#define FR_W(W_)                                                               \
  case W_:                                                                     \
    if constexpr (F > 1 && W_ > FR_SPOP_GRADT_FIELDS_WMAX)                     \
      return hipErrorInvalidValue;                                             \
    else if constexpr (F > 1) spop_launch_gradt<T, EPI, W_, DG, F>(g, sp, s);  \
    else if constexpr (EPI == EPI_GRADTF) return hipErrorInvalidValue;         \
    else if (g.D == 3) spop_launch_gradt<T, EPI, W_, 3, F>(g, sp, s);          \
    else spop_launch_gradt<T, EPI, W_, 2, F>(g, sp, s);                        \
    break;
    FR_SPOP_WIDTHS(FR_W)
#undef FR_W
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int EPI, int F>
hipError_t spop_launch_t(const GemmArgs &g, const SparseOp &sp, int batch, hipStream_t s) {
  switch (sp.width) {
#define FR_W(W_) \
  case W_: spop_launch_w<T, EPI, W_, F>(g, sp, batch, s); break;
    FR_SPOP_WIDTHS(FR_W)
#undef FR_W
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Launch with F fields per thread (F = 1, or the field count with
// g.N == F * g.ld).
template <int F>
hipError_t launch_spop_f(int prec, int epi, const GemmArgs &g, const SparseOp &sp, int batch,
                         hipStream_t s) {
  if (F > 1 && g.N != (int64_t)F * g.ld) return hipErrorInvalidValue;
  if (epi == EPI_ADDT) {
    // the D batch slices are looped inside the kernel
    if (batch != 1 || prec != PREC_F64) return hipErrorInvalidValue;
    return spop_addt_t<F>(g, sp, s);
  }
  if (epi == EPI_GRADT) {
    if (batch != 1) return hipErrorInvalidValue;
    if (prec == PREC_F64) return spop_gradt_t<double, F>(g, sp, s);
    if (prec == PREC_F32) return spop_gradt_t<float, F>(g, sp, s);
    return hipErrorInvalidValue;
  }
  if (epi == EPI_GRADTF) {
    if constexpr (F == 1) {
      return hipErrorInvalidValue;
    } else {
      if (batch != 1) return hipErrorInvalidValue;
      if (prec == PREC_F64) return spop_gradt_t<double, F, EPI_GRADTF>(g, sp, s);
      if (prec == PREC_F32) return spop_gradt_t<float, F, EPI_GRADTF>(g, sp, s);
      return hipErrorInvalidValue;
    }
  }
  if (epi == EPI_TFVJP) {
    if constexpr (F == 1) {
      return hipErrorInvalidValue;
    } else {
      if (batch != 1 || prec != PREC_F64) return hipErrorInvalidValue;
      return spop_gradt_t<double, F, EPI_TFVJP>(g, sp, s);
    }
  }
  if (prec == PREC_F64) {
    switch (epi) {
      case EPI_STORE: return spop_launch_t<double, EPI_STORE, F>(g, sp, batch, s);
      case EPI_NEGDIV: return spop_launch_t<double, EPI_NEGDIV, F>(g, sp, batch, s);
      case EPI_RK: return spop_launch_t<double, EPI_RK, F>(g, sp, batch, s);
      case EPI_ADD: return spop_launch_t<double, EPI_ADD, F>(g, sp, batch, s);
      case EPI_RKADJ:
        if (batch != 1 || !g.acc || !g.stage || !g.dt || !g.rcpdjac) return hipErrorInvalidValue;
        return spop_launch_t<double, EPI_RKADJ, F>(g, sp, batch, s);
    }
  } else if (prec == PREC_F32) {
    switch (epi) {
      case EPI_STORE: return spop_launch_t<float, EPI_STORE, F>(g, sp, batch, s);
      case EPI_NEGDIV: return spop_launch_t<float, EPI_NEGDIV, F>(g, sp, batch, s);
      case EPI_RK: return spop_launch_t<float, EPI_RK, F>(g, sp, batch, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spop_fields4(int prec, int epi, const GemmArgs &g, const SparseOp &sp,
                               int batch, hipStream_t s);
hipError_t launch_spop_fields5(int prec, int epi, const GemmArgs &g, const SparseOp &sp,
                               int batch, hipStream_t s);

}  // namespace fr
