// Gravitational acceleration on the cell faces (Sec. 2.1, Eq. gradient):
// g = -grad Phi, its face-normal component the difference of the potential
// in the two cells that share the face over the distance of their centroids
// projected on the face normal -- radial faces d = a_{i+1} - a_i; theta
// faces r_i (theta_{j+1} - theta_j), z faces z_{j+1} - z_j; azimuthal faces
// r_i sin(theta_j) dphi (spherical) or R_i dphi (cylindrical).  A boundary
// face takes the ghost cell's potential, the second solve's Dirichlet value
// -Theta transformed back to phi; a face lying on a pole has zero area and
// carries g = 0 (its inverse distance is stored as 0).
//
// One thread per cell (phi fastest, so every read and write is coalesced)
// writes the lower radial, lower theta/z and upper azimuthal face of its
// cell, and the cells of the last radial or theta/z layer also the upper
// boundary face.  HBM-bound: 8 bytes read and 24 written per cell.
#include "smg_internal.h"
#include "vec.h"

namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) k_accel(AccelArgs A) {
  const auto phi = gbl(A.phi);
  const auto gpot = gbl(A.gpot);
  const int na = A.na, nb = A.nb, nphi = A.nphi;
  const size_t n = (size_t)na * nb * nphi;
  const size_t plane = (size_t)nb * nphi;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % nphi);
    const size_t ij = t / nphi;
    const int j = (int)(ij % nb), i = (int)(ij / nb);
    const double c = phi[t];
    // radial faces (face i - 1/2 at index t; face na - 1/2 one plane further)
    const double alo = i > 0 ? phi[t - plane] : -gpot[(size_t)j * nphi + k];
    A.ga[t] = (alo - c) * A.inv_da[i];
    if (i == na - 1) {
      const double ahi = -gpot[(size_t)(A.g_ahi + j) * nphi + k];
      A.ga[t + plane] = (c - ahi) * A.inv_da[na];
    }
    // theta / z faces (face j - 1/2; face nb - 1/2 for the last layer)
    const double bm = A.sph ? A.inv_ra[i] : 1.0;
    const size_t tb = ((size_t)i * (nb + 1) + j) * nphi + k;
    const double blo = j > 0 ? phi[t - nphi] : (A.g_blo >= 0 ? -gpot[(size_t)(A.g_blo + i) * nphi + k] : c);
    A.gb[tb] = (blo - c) * A.inv_db[j] * bm;
    if (j == nb - 1) {
      const double bhi = A.g_bhi >= 0 ? -gpot[(size_t)(A.g_bhi + i) * nphi + k] : c;
      A.gb[tb + nphi] = (c - bhi) * A.inv_db[nb] * bm;
    }
    // azimuthal face k + 1/2 (periodic)
    const double cn = phi[t - k + (k + 1 == nphi ? 0 : k + 1)];
    A.gp[t] = (c - cn) * A.inv_ra[i] * A.inv_sb[j] * A.inv_dphi;
  }
}

}  // namespace

namespace smgk {

hipError_t accel(const AccelArgs& a, hipStream_t st) {
  const size_t n = (size_t)a.na * a.nb * a.nphi;
  if (n == 0) return hipSuccess;
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_accel, dim3((unsigned)g), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace smgk
