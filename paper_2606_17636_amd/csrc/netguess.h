// Launchers of the learned-guess steps inside a solve (netguess.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace smgg {
// images: 0 = re(m=0); 2m-1 = re(m), 2m = im(m) for m = 1..m_max (n_img = 2 m_max + 1)
// sc[4 k + (0, 1, 2, 3)] = (s_f, s_d, s_u, s_o) per image: RMS of f_t, of
// f_t - f_prev, of u_prev, and the output scale s_o: the RMS of
// u_prev - u_prev2 (uprev2 given) or s_u s_d / s_f
// part: scratch of scales_partial_doubles(n_img) doubles
size_t scales_partial_doubles(int n_img);
hipError_t scales(const double2* f, const double2* fprev, const double2* uprev, const double2* uprev2, int plane, int n_img,
                  double* part, double* sc, hipStream_t st);
// uprev2: the solution two steps back (channel 6 = (uprev - uprev2) / s_o), or null
hipError_t assemble(const double2* f, const double2* fprev, const double2* uprev, const double2* uprev2, const double* sc,
                    int na, int nb, int n_img, float* x, hipStream_t st);
// base = uprev + (uprev - uprev2 if uprev2; not on static parts), cand = base + s_o y
// (also into cand2 when given: the copy the judge smooths)
hipError_t candidate(const double2* uprev, const double2* uprev2, const float* y, const double* sc, int plane, int m_max,
                     double2* cand, double2* base, hipStream_t st, double2* cand2 = nullptr);
// per mode: u = cand where pc's norm is below pu's, else base (recomputed; u left as it is with uprev null)
hipError_t select(const double* pc, const double* pu, int nblk, const double2* cand, const double2* uprev,
                  const double2* uprev2, const double* sc, double2* u, int plane, int m_max, int* used, hipStream_t st);
hipError_t record(const float* x, const double2* u, const double2* uprev, const double2* uprev2, const double* sc,
                  int plane, int n_img, int* count, int capacity, float* samples, hipStream_t st);
// warm start from the last k solutions (n values; hist[0..kept-1] the kept older ones, newest
// first; k <= kept + 1): from value lo on, u <- the polynomial extrapolation through them
// (2 u - h0, 3 u - 3 h0 + h1, 4 u - 6 h0 + 4 h1 - h2); u's old value goes into hist[kept - 1]
// (the caller's ring of slots then makes that slot the newest)
hipError_t extrapolate(double2* u, double2* const* hist, int kept, size_t n, size_t lo, int k, hipStream_t st);
}  // namespace smgg
