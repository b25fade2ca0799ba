// Device-side views used by the discrete Green's function construction
// (dgf.hip) and its host driver.
#pragma once

#include "smg_internal.h"

struct DgfConst {
  int sph;            // 1 spherical, 0 cylindrical
  int n_phi;
  int n_g;            // number of boundary ghost cells
  double G;
  const double* cosk;  // cos(2 pi k / n_phi), k < n_phi
  const double* s2;    // s_m^2 indexed by azimuthal index m
};

// Auxiliary boxes (one per source ghost) and the continued-axis tables they
// index into (local index = global index - off).
struct AuxBoxes {
  const int *i_lo, *i_hi, *j_lo, *j_hi;
  const int *e_alo, *e_blo, *e_bhi;    // 0 Dirichlet, 1 pole, 2 Neumann
  int offA, offB;
  const double *centA, *faceA, *upA, *dnA, *RA, *PA, *nfA;
  const double *centB, *upB, *dnB, *PB;
  const int *gi, *gj;                   // ghost global indices
  const double *ga, *gb, *gdv;          // ghost coordinates and 3D volumes
};

// Extended domain shared by all sources (level-0 geometry of its hierarchy).
struct ExtBox {
  int na, nb;
  int e_blo, e_bhi;                     // 0 Dirichlet, 1 pole
  const double *centA, *centB;          // na+2, nb+2 (local, with ghosts)
  const double* RA;                     // na interior metric factor
  double face0;                         // inner (Neumann) face
  double nfA;                           // face area / volume of the first cell
  double upA_last, dnB_first, upB_last; // couplings toward the Dirichlet rings
  const int* cell;                      // box cell index of every ghost
  const double *ga, *gb, *gdv;
};

__device__ double kernel_sum(const DgfConst& K, int m, double a, double b, double as, double bs);
__device__ double kernel_dr_sum(const DgfConst& K, int m, double a, double b, double as, double bs);

namespace smgk {
hipError_t dgf_aux(const DgfConst& K, const AuxBoxes& X, const int* modes, int n_modes, double* out, double tol,
                   int max_sweeps, double* resid, int max_n1, int max_n2, hipStream_t st);
hipError_t dgf_ext_rhs(const DgfConst& K, const ExtBox& E, const int* pmode, const int* src0, const int* src1,
                       int nplanes, double2* f, hipStream_t st);
hipError_t dgf_ext_extract(const ExtBox& E, int n_g, const int* ptab, const int* src0, const int* src1, int nplanes,
                           const double2* u, double* out, hipStream_t st);
}  // namespace smgk
