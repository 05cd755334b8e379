// Host-side set-up of the FR operators, metric terms and pair tables.
//
// Runs once per context in FP64 (long double for the Vandermonde solve), as
// the paper's set-up phase does (section 3, operator matrices built once on
// the host).  Nothing here touches the device.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace fr {

struct SetupError : std::runtime_error {
  int status;
  SetupError(int s, const std::string &m) : std::runtime_error(m), status(s) {}
};

enum { ET_QUAD = 0, ET_TRI = 1, ET_HEX = 2 };
// Correction-function schemes (members of the VCJH family): DG, SD, HU.
enum { CORR_DG = 0, CORR_SD = 1, CORR_HU = 2 };

// Reference element of one (type, order): points and the Appendix A
// operators, all row-major.
struct RefOps {
  int etype = 0, p = 0, corr = CORR_DG, ndims = 0, nupts = 0, nfpts = 0, nfaces = 0, nfp_face = 0;
  std::vector<double> upts, fpts, fnorm;   // [n][ndims]
  std::vector<int> fface;                  // face of each flux point
  std::vector<double> fweight;             // omega_sigma: face quadrature weight
  std::vector<double> W;                   // integral of l_rho (quadrature weights)
  // Appendix A operators (row-major, dims in comments)
  std::vector<double> M0;                  // Nf x Nu          l_rho(x^f_sigma)
  std::vector<double> M3;                  // Nu x Nf          div g_sigma at x^u_rho
  std::vector<double> M4p;                 // D Nu x Nu        M4 - M6 M0
  std::vector<double> M6;                  // D Nu x Nf        n~_sigma,i div g_sigma
  std::vector<double> M1p;                 // Nu x D Nu        M1 - M3 M2
  std::vector<double> M1, M2, M4;          // kept for tests of the identities
};

// corr: CORR_DG for every element type; CORR_SD and CORR_HU for quads and
// hexes only (SetupError status 3 otherwise).
RefOps build_ref(int etype, int p, int corr = CORR_DG);

// Metric terms of one element block, device layout ([component][rho][ld]).
struct BlockGeom {
  int64_t nelem = 0, ld = 0;
  std::vector<double> smat;     // [D][D][Nu][ld]  S = adj J = J J^-1, (i=ref, j=phys)
  std::vector<double> rcpdjac;  // [Nu][ld]        1/J
  std::vector<double> wdjac;    // [Nu][ld]        W_rho J (integration weights)
  std::vector<double> xu;       // [nelem][Nu][D]  physical solution points
  std::vector<double> xf;       // [nelem][Nf][D]  physical flux points
  std::vector<double> fnhat;    // [nelem][Nf][D]  unit physical outward normal
  std::vector<double> fmag;     // [nelem][Nf]     J^(f) n^(f) = |S^T n~|
  double hmin = 0;              // smallest element extent (pairing tolerance)
};

BlockGeom build_geom(const RefOps &ref, int geom_order, int64_t nelem, const double *nodes,
                     int64_t ld);

struct FacePairIn {
  int lblock, lface; int64_t lelem;
  int rblock, rface; int64_t relem;
  double shift[3];
};

// Flux-point pair table, sorted for coalesced access on the L side.
struct PairTable {
  int64_t n = 0;
  std::vector<int32_t> lblk, rblk;   // block of each side
  std::vector<int64_t> lidx, ridx;   // sigma * nvars * ld + n within the block's U^f
  std::vector<double> nrm;           // [D][n] unit normal of the L side
  std::vector<double> magL, magR;    // J^(f) n^(f) on each side
};

// A face on the domain boundary (Appendix C: one flux point per boundary
// interface point, with a boundary type).
struct BcFaceIn {
  int block, face; int64_t elem; int bc;
};

// Boundary flux-point table, sorted like the pair table's L side.
struct BcTable {
  int64_t n = 0;
  std::vector<int32_t> blk, bc;      // block and boundary condition of each point
  std::vector<int64_t> idx;          // sigma * nvars * ld + n within the block's U^f
  std::vector<double> nrm;           // [D][n] outward unit normal
  std::vector<double> mag;           // J^(f) n^(f)
};

// Pairs every flux point of the face pairs; flux points of boundary faces go
// to `bct` (bcfaces may be null with nbcfaces = 0).  Every flux point must be
// paired or on a boundary face exactly once.
PairTable build_pairs(const std::vector<RefOps> &refs, const std::vector<BlockGeom> &geoms,
                      const std::vector<int> &block_ref, int ndims, int nvars,
                      const FacePairIn *pairs, int64_t npairs, const BcFaceIn *bcfaces,
                      int64_t nbcfaces, int nbcs, BcTable *bct);

int nnodes_of(int etype, int geom_order);

}  // namespace fr
