// Host-side FP64 expansion operators (real solid-harmonic basis).
//
// Expansions follow the multipole / local factorisation of the kernel in
// Sec. 2.3 (Eq. (14)).  Complex solid harmonics, for m >= 0:
//   R_n^m(r) = r^n P_n^m(cos t) e^{i m f} / (n+m)!          (regular)
//   I_n^m(r) = (n-m)! P_n^m(cos t) e^{i m f} / r^{n+1}      (irregular)
// with P_n^m the associated Legendre function without the Condon-Shortley
// phase, and for m < 0: X_n^{-m} = (-1)^m conj(X_n^m).  With these,
//   1/|x - y|   = sum_{n,m} conj(R_n^m(y)) I_n^m(x)             (|y| < |x|)
//   R_n^m(a+b)  = sum_{j,k} R_j^k(a) R_{n-j}^{m-k}(b)
//   I_n^m(D+y)  = sum_{j,k} (-1)^j conj(R_j^k(y)) I_{n+j}^{m+k}(D) (|y| < |D|)
// from which:
//   P2M  M_n^m  = sum_i q_i conj(R_n^m(x_i - c))
//   M2M  M'_n^m = sum_{j,k} M_j^k conj(R_{n-j}^{m-k}(c - c'))
//   M2L  L_j^k  = (-1)^{j+k} sum_{n,m} M_n^m I_{n+j}^{m-k}(c_L - c_M)
//   L2L  L'_j^k = sum_{n,m} L_n^m R_{n-j}^{m-k}(c' - c)
//   L2P  phi(x) = sum_{j,k} L_j^k R_j^k(x - c),  g = -grad(phi).
// Expansions are stored scaled by the box width w of their level,
// Mt_n = M_n / w^n and Lt_n = L_n w^{n+1}, which makes every translation
// matrix independent of the level.  Real storage: degree n occupies
// [n^2, (n+1)^2): m = 0 real part, then (re, im) of m = 1..n.
#pragma once

#include <complex>
#include <vector>

namespace grav {

using cd = std::complex<double>;

inline int ridx(int n, int m, int part) { return m == 0 ? n * n : n * n + 2 * m - 1 + part; }

// Solid harmonics for n < P, 0 <= m <= n, stored at [n * P + m].
void solid_regular(double x, double y, double z, int P, std::vector<cd> &R);
void solid_irregular(double x, double y, double z, int P, std::vector<cd> &I);

// Signed-m access with the X^{-m} = (-1)^m conj(X^m) rule; zero outside |m| <= n.
cd sh_get(const std::vector<cd> &A, int P, int n, int m);

// Dense real operator matrices, row-major [rows = out coefficient][cols = in],
// with row and column stride `ld` (>= P*P, extra entries zero).
void m2m_matrix(int P, const double delta[3], int ld, double *out);
void l2l_matrix(int P, const double delta[3], int ld, double *out);
void m2l_matrix(int P, const double d[3], int ld, double *out);

// Lattice P2M: for a leaf of b^3 cells with q^3 Gauss points each, the
// scaled ME of unit density in cell v is column v.  Out: [b^3][ld], the
// coefficients of cell v contiguous.  h = cell edge, positions in units of
// the leaf edge b*h relative to the leaf centre.
void p2m_lattice(int P, int b, int q, double h, int ld, double *out);

// Near field on the lattice: for targets at the b^3 cell centres of a leaf and
// the Gauss points (q = 1 or 2 per axis) of the b^3 cells of the leaf at
// offset d (d in {-1, 0, 1}^3, index nb = (dx+1) + 3 (dy+1) + 9 (dz+1)), the
// matrix that maps cell densities to (phi, gx, gy, gz) with phi = sum w / r and
// g_a = sum w u_a / r^3, u = target - source, in cell units (h = 1, unit
// density: w = 1/8 per Gauss point for q = 2, 1 for q = 1).  Pairs with
// r^2 <= coincident_r2 are left out.  Layout: out[nb][4 t + comp][s], t and s
// cell indices x fastest.  The direct sum over the same pairs gives the same
// values; the matrices depend only on (b, q) because both point sets sit on
// the lattice.
void near_lattice(int b, int q, double coincident_r2, double *out);

}  // namespace grav
