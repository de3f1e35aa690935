// Regular solid harmonics on the device: the real coefficient order of the
// expansions and the recurrences shared by the point kernels of the forward
// pass and its transpose.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace grav {

// Real index of the regular harmonic / coefficient (n, m): the real part
// (order 0, or part 0 of order m > 0) or the imaginary part (part 1).
__device__ __forceinline__ int harm_index(int n, int m, int part)
{
    return m == 0 ? n * n : n * n + 2 * m - 1 + part;
}

// The regular solid harmonics R_n^m(u), n < P, in the coefficients' real
// order (the recurrences of l2p_eval), written to h[k * CS].
__device__ inline void regular_harmonics(int P, double x, double y, double z, double *h, int CS)
{
    const double r2 = x * x + y * y + z * z;
    double mmr = 1.0, mmi = 0.0;
    for (int m = 0; m < P; ++m) {
        if (m > 0) {
            const double s = 1.0 / (2.0 * m);
            const double nr = (x * mmr - y * mmi) * s;
            const double ni = (x * mmi + y * mmr) * s;
            mmr = nr;
            mmi = ni;
        }
        double p1r = 0.0, p1i = 0.0, p2r = 0.0, p2i = 0.0;
        for (int n = m; n < P; ++n) {
            double Rr, Ri;
            if (n == m) {
                Rr = mmr;
                Ri = mmi;
            } else if (n == m + 1) {
                Rr = z * p1r;
                Ri = z * p1i;
            } else {
                const double f = 1.0 / (double)((n - m) * (n + m));
                Rr = ((2.0 * n - 1.0) * z * p1r - r2 * p2r) * f;
                Ri = ((2.0 * n - 1.0) * z * p1i - r2 * p2i) * f;
            }
            p2r = p1r;
            p2i = p1i;
            p1r = Rr;
            p1i = Ri;
            h[harm_index(n, m, 0) * CS] = Rr;
            if (m > 0)
                h[harm_index(n, m, 1) * CS] = Ri;
        }
    }
}

// Multipole basis of a unit point mass at u (leaf widths from the leaf
// centre), in the coefficients' real order (the lattice P2M's basis):
// R_n^0, and Re R_n^m, -Im R_n^m for m > 0 (the conjugate harmonic).
// acc[t] += sum_k basis_k(u) a[t * stride + k] for t < nm (its transpose:
// the derivative of the leaf expansions with respect to the mass).
template <int MT>
__device__ inline void multipole_basis_dot(int P, double x, double y, double z, const double *a, int64_t stride,
                                           int nm, double (&acc)[MT])
{
    const double r2 = x * x + y * y + z * z;
    double mmr = 1.0, mmi = 0.0;
    for (int m = 0; m < P; ++m) {
        if (m > 0) {
            const double s = 1.0 / (2.0 * m);
            const double nr = (x * mmr - y * mmi) * s;
            const double ni = (x * mmi + y * mmr) * s;
            mmr = nr;
            mmi = ni;
        }
        double p1r = 0.0, p1i = 0.0, p2r = 0.0, p2i = 0.0;
        for (int n = m; n < P; ++n) {
            double Rr, Ri;
            if (n == m) {
                Rr = mmr;
                Ri = mmi;
            } else if (n == m + 1) {
                Rr = z * p1r;
                Ri = z * p1i;
            } else {
                const double f = 1.0 / (double)((n - m) * (n + m));
                Rr = ((2.0 * n - 1.0) * z * p1r - r2 * p2r) * f;
                Ri = ((2.0 * n - 1.0) * z * p1i - r2 * p2i) * f;
            }
            p2r = p1r;
            p2i = p1i;
            p1r = Rr;
            p1i = Ri;
            const int kr = harm_index(n, m, 0);
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                if (t >= nm)
                    break;
                acc[t] += Rr * a[t * stride + kr];
                if (m > 0)
                    acc[t] -= Ri * a[t * stride + kr + 1];
            }
        }
    }
}

}  // namespace grav
