// Host-side FP64 expansion operators; see operators.hpp for the formulas.
#include "operators.hpp"

#include <cmath>
#include <cstring>

namespace grav {

void solid_regular(double x, double y, double z, int P, std::vector<cd> &R)
{
    R.assign((size_t)P * P, cd(0.0, 0.0));
    const double r2 = x * x + y * y + z * z;
    const cd xy(x, y);
    R[0] = 1.0;
    for (int m = 0; m < P; ++m) {
        if (m > 0)  // R_m^m = (x + iy) / (2m) R_{m-1}^{m-1}
            R[m * P + m] = xy / (2.0 * m) * R[(m - 1) * P + (m - 1)];
        if (m + 1 < P)  // R_{m+1}^m = z R_m^m
            R[(m + 1) * P + m] = z * R[m * P + m];
        for (int n = m + 2; n < P; ++n)  // Legendre three-term recurrence in n
            R[n * P + m] = ((2.0 * n - 1.0) * z * R[(n - 1) * P + m] - r2 * R[(n - 2) * P + m]) /
                           (double)((n - m) * (n + m));
    }
}

void solid_irregular(double x, double y, double z, int P, std::vector<cd> &I)
{
    I.assign((size_t)P * P, cd(0.0, 0.0));
    const double r2 = x * x + y * y + z * z;
    const double ir2 = 1.0 / r2;
    const cd xy(x, y);
    I[0] = std::sqrt(ir2);
    for (int m = 0; m < P; ++m) {
        if (m > 0)  // I_m^m = (2m - 1)(x + iy)/r^2 I_{m-1}^{m-1}
            I[m * P + m] = (2.0 * m - 1.0) * xy * ir2 * I[(m - 1) * P + (m - 1)];
        if (m + 1 < P)  // I_{m+1}^m = (2m + 1) z / r^2 I_m^m
            I[(m + 1) * P + m] = (2.0 * m + 1.0) * z * ir2 * I[m * P + m];
        for (int n = m + 2; n < P; ++n)
            I[n * P + m] = ((2.0 * n - 1.0) * z * I[(n - 1) * P + m] -
                            (double)((n + m - 1) * (n - m - 1)) * I[(n - 2) * P + m]) *
                           ir2;
    }
}

cd sh_get(const std::vector<cd> &A, int P, int n, int m)
{
    if (n < 0 || n >= P || m > n || -m > n)
        return cd(0.0, 0.0);
    if (m >= 0)
        return A[n * P + m];
    const cd v = std::conj(A[n * P + (-m)]);
    return ((-m) & 1) ? -v : v;
}

// Turn a complex linear map out_j^k = sum_{n, m=-n..n} c(j,k,n,m) in_n^m,
// whose input obeys in_n^{-m} = (-1)^m conj(in_n^m), into a real matrix
// acting on the real storage.
template <class F>
static void real_matrix(int P, int ld, double *out, F c)
{
    std::memset(out, 0, sizeof(double) * (size_t)ld * ld);
    for (int j = 0; j < P; ++j)
        for (int k = 0; k <= j; ++k)
            for (int n = 0; n < P; ++n)
                for (int m = 0; m <= n; ++m) {
                    const cd c1 = c(j, k, n, m);
                    double *row_re = out + (size_t)ridx(j, k, 0) * ld;
                    double *row_im = k > 0 ? out + (size_t)ridx(j, k, 1) * ld : nullptr;
                    if (m == 0) {
                        row_re[ridx(n, 0, 0)] += c1.real();
                        if (row_im)
                            row_im[ridx(n, 0, 0)] += c1.imag();
                    } else {
                        cd c2 = c(j, k, n, -m);
                        if (m & 1)
                            c2 = -c2;
                        const cd sp = c1 + c2, sm = c1 - c2;
                        row_re[ridx(n, m, 0)] += sp.real();
                        row_re[ridx(n, m, 1)] += -sm.imag();
                        if (row_im) {
                            row_im[ridx(n, m, 0)] += sp.imag();
                            row_im[ridx(n, m, 1)] += sm.real();
                        }
                    }
                }
}

// delta: child centre minus parent centre, in parent-width units (+-1/4).
void m2m_matrix(int P, const double delta[3], int ld, double *out)
{
    std::vector<cd> Rd;
    solid_regular(delta[0], delta[1], delta[2], P, Rd);
    std::vector<double> half(P);
    for (int j = 0; j < P; ++j)
        half[j] = std::ldexp(1.0, -j);
    // out (n, m) <- in (j, k): (1/2)^j conj(R_{n-j}^{m-k}(delta))
    real_matrix(P, ld, out, [&](int n, int m, int j, int k) -> cd {
        if (j > n)
            return cd(0.0, 0.0);
        return half[j] * std::conj(sh_get(Rd, P, n - j, m - k));
    });
}

// delta: child centre minus parent centre, in parent-width units.
void l2l_matrix(int P, const double delta[3], int ld, double *out)
{
    std::vector<cd> Rd;
    solid_regular(delta[0], delta[1], delta[2], P, Rd);
    real_matrix(P, ld, out, [&](int j, int k, int n, int m) -> cd {
        if (n < j)
            return cd(0.0, 0.0);
        return std::ldexp(1.0, -(j + 1)) * sh_get(Rd, P, n - j, m - k);
    });
}

// d: target-box centre minus source-box centre in box units.
void m2l_matrix(int P, const double d[3], int ld, double *out)
{
    const int P2 = 2 * P;
    std::vector<cd> Id;
    solid_irregular(d[0], d[1], d[2], P2, Id);
    real_matrix(P, ld, out, [&](int j, int k, int n, int m) -> cd {
        const cd v = sh_get(Id, P2, n + j, m - k);
        return ((j + k) & 1) ? -v : v;
    });
}

void p2m_lattice(int P, int b, int q, double h, int ld, double *out)
{
    double gx[2], gw[2];
    int nq = 1;
    gx[0] = 0.0;
    gw[0] = 1.0;
    if (q == 2) {
        nq = 2;
        gx[0] = -0.5 / std::sqrt(3.0);
        gx[1] = 0.5 / std::sqrt(3.0);
        gw[0] = gw[1] = 0.5;
    }
    const double vol = h * h * h;
    std::memset(out, 0, sizeof(double) * (size_t)b * b * b * ld);
    std::vector<cd> R;
    for (int kz = 0; kz < b; ++kz)
        for (int ky = 0; ky < b; ++ky)
            for (int kx = 0; kx < b; ++kx) {
                double *col = out + (size_t)((kz * b + ky) * b + kx) * ld;
                for (int a = 0; a < nq; ++a)
                    for (int bb = 0; bb < nq; ++bb)
                        for (int c = 0; c < nq; ++c) {
                            const double u = ((kx + 0.5 + gx[c]) / b) - 0.5;
                            const double v = ((ky + 0.5 + gx[bb]) / b) - 0.5;
                            const double w = ((kz + 0.5 + gx[a]) / b) - 0.5;
                            const double wt = vol * gw[a] * gw[bb] * gw[c];
                            solid_regular(u, v, w, P, R);
                            for (int n = 0; n < P; ++n) {
                                col[ridx(n, 0, 0)] += wt * R[n * P].real();
                                for (int m = 1; m <= n; ++m) {
                                    const cd cr = std::conj(R[n * P + m]);
                                    col[ridx(n, m, 0)] += wt * cr.real();
                                    col[ridx(n, m, 1)] += wt * cr.imag();
                                }
                            }
                        }
            }
}

void near_lattice(int b, int q, double coincident_r2, double *out)
{
    const int b3 = b * b * b;
    const double go = 0.5 / std::sqrt(3.0);
    std::memset(out, 0, sizeof(double) * 27 * (size_t)4 * b3 * b3);
    for (int nb = 0; nb < 27; ++nb) {
        const int d[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, nb / 9 - 1};
        double *m = out + (size_t)nb * 4 * b3 * b3;
        for (int t = 0; t < b3; ++t) {
            const int tc[3] = {t % b, (t / b) % b, t / (b * b)};
            for (int sidx = 0; sidx < b3; ++sidx) {
                const int sc[3] = {sidx % b, (sidx / b) % b, sidx / (b * b)};
                double c[3];
                for (int a = 0; a < 3; ++a)
                    c[a] = (double)(tc[a] - sc[a] - d[a] * b);  // target centre - source centre
                double acc[4] = {0, 0, 0, 0};
                const int ng = q == 2 ? 8 : 1;
                for (int gp = 0; gp < ng; ++gp) {
                    double u[3];
                    for (int a = 0; a < 3; ++a)
                        u[a] = q == 2 ? c[a] - (((gp >> a) & 1) ? go : -go) : c[a];
                    const double r2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                    if (!(r2 > coincident_r2))
                        continue;
                    const double w = q == 2 ? 0.125 : 1.0;
                    const double ri = 1.0 / std::sqrt(r2);
                    acc[0] += w * ri;
                    for (int a = 0; a < 3; ++a)
                        acc[1 + a] += w * ri * ri * ri * u[a];
                }
                for (int comp = 0; comp < 4; ++comp)
                    m[(size_t)(4 * t + comp) * b3 + sidx] = acc[comp];
            }
        }
    }
}

}  // namespace grav
