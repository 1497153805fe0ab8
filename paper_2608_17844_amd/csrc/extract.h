// Device-side port-quantity extraction (internal).
#pragma once

#include "common.h"

namespace mbt {

// Inverse of the n x n array A (overwritten) into out, Gauss-Jordan with partial pivoting.
// colbuf: n complex; piv: n ints; flag: 1 int; out (n x n, not overlapping A) serves as
// workspace until the result is written.  Throws on a singular matrix.
void gj_inverse(double2* A, double2* out, int n, double2* colbuf, int* piv, int* flag, hipStream_t s);
// S = I - 2 z0 (Zp + z0 I)^{-1}; work: n*n complex scratch.
void s_matrix(const double2* Zp, double2* S, double2* work, int n, double z0, double2* colbuf, int* piv, int* flag,
              hipStream_t s);
// The same S with every workspace on the device (colbuf n complex, piv and src
// n ints, flag 1 int) and host_flag one pinned int: no host buffers.
void s_matrix_dev_perm(const double2* Zp, double2* S, double2* work, int n, double z0, double2* colbuf, int* piv,
                       int* src, int* flag, int* host_flag, hipStream_t s);
// Center-element active impedance, ARC and wave-excited ARC for nscan directions (device arrays).
void scans(const Geom& g, double k, const double2* Zp, const double2* S, int c, const double* theta, const double* phi,
           int nscan, double z0, double2* Za, double2* G, double2* Gw, hipStream_t s);

// Phased voltage excitation of every gap (R columns, layout [n][r]):
// V = w_i exp(-j k (x_e u + y_e v)) at the port bases of each element e.
void scan_voltages(const Geom& g, double k, const double* theta, const double* phi, int R, double2* V,
                   hipStream_t s);
// Center-element active impedance V_c / I_p,c and ARC from the gap currents Ip (P x nscan, column-major).
void scan_active(const Geom& g, double k, const double2* Ip, int nscan, int c, const double* theta,
                 const double* phi, double z0, double2* Za, double2* G, hipStream_t s);

}  // namespace mbt
