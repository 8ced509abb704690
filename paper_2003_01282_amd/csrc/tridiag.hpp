// FP64 symmetric tridiagonal eigensolver for the Gauss rule (paper §3.1,
// eq. "quadratic": nodes are the eigenvalues of the Lanczos matrix T, weights
// the squared first components of its normalized eigenvectors, following
// Golub and Welsch).  Only the first row of the eigenvector matrix is carried.
//
// Implicit symmetric QR steps with the Wilkinson shift (Golub and Van Loan,
// "Matrix Computations", the implicit symmetric QR step), bulge chasing with
// Givens rotations, deflation of negligible off-diagonals from the bottom.
// The arrays are accessed through a stride so callers can keep one matrix
// per thread in LDS with conflict-free interleaving.
#pragma once

#include <hip/hip_runtime.h>

namespace slaq {

// d[k*stride], e[k*stride] (e couples k and k+1), u[k*stride] = first row of U.
// On return d holds the eigenvalues and u the first components.  Returns the
// number of sweeps, or -1 if the iteration cap was hit.
__device__ inline int tridiag_eig_first_row(double* d, double* e, double* u, int n, int stride) {
    for (int k = 0; k < n; ++k) u[k * stride] = k == 0 ? 1.0 : 0.0;
    if (n <= 1) return 0;
    const double eps = 2.220446049250313e-16;
    int sweeps = 0;
    const int cap = 60 * n;
    int hi = n - 1;
    while (hi > 0) {
        const double dh = d[hi * stride], dl = d[(hi - 1) * stride];
        const double eh = e[(hi - 1) * stride];
        if (fabs(eh) <= eps * (fabs(dh) + fabs(dl)) || fabs(eh) < 1e-300) {
            e[(hi - 1) * stride] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0) {
            const double el = e[(lo - 1) * stride];
            if (fabs(el) <= eps * (fabs(d[(lo - 1) * stride]) + fabs(d[lo * stride])) || fabs(el) < 1e-300) {
                e[(lo - 1) * stride] = 0.0;
                break;
            }
            --lo;
        }
        if (++sweeps > cap) return -1;
        // Wilkinson shift from the trailing 2x2 block
        const double delta = 0.5 * (dl - dh);
        const double r = hypot(delta, eh);
        const double denom = delta + (delta >= 0.0 ? r : -r);
        const double mu = dh - eh * eh / denom;
        double x = d[lo * stride] - mu;
        double z = e[lo * stride];
        // the bulge chase carries d[k], e[k] and u[k] in registers from one
        // rotation to the next (each sweep finalizes index k as it moves on);
        // only the next index is loaded, so the loads do not sit on the
        // dependent chain of the rotations
        double a = d[lo * stride], b = e[lo * stride], u0 = u[lo * stride];
        for (int k = lo; k < hi; ++k) {
            const double dd = d[(k + 1) * stride];
            const double u1 = u[(k + 1) * stride];
            const double en = k + 1 < hi ? e[(k + 1) * stride] : 0.0;
            // rotation with s*x + c*z = 0: the larger of |c|, |s| positive,
            // both from one reciprocal square root of x^2 + z^2 (no division;
            // a ratio-based form guards squares that would over- or underflow)
            double c, s;
            const double r2 = x * x + z * z;
            if (z == 0.0) {
                c = 1.0;
                s = 0.0;
            } else if (r2 > 1e-290 && r2 < 1e290) {
                const double ri = rsqrt(r2);
                if (fabs(z) > fabs(x)) {
                    s = fabs(z) * ri;
                    c = -x * copysign(ri, z);
                } else {
                    c = fabs(x) * ri;
                    s = -z * copysign(ri, x);
                }
            } else if (fabs(z) > fabs(x)) {
                const double tau = -x / z;
                s = rsqrt(1.0 + tau * tau);
                c = s * tau;
            } else {
                const double tau = -z / x;
                c = rsqrt(1.0 + tau * tau);
                s = c * tau;
            }
            if (k > lo) e[(k - 1) * stride] = c * x - s * z;
            const double cc = c * c, ss = s * s, cs = c * s;
            d[k * stride] = a * cc - 2.0 * b * cs + dd * ss;
            const double a_next = a * ss + 2.0 * b * cs + dd * cc;
            const double bn = (a - dd) * cs + b * (cc - ss);
            u[k * stride] = c * u0 - s * u1;
            const double u_next = s * u0 + c * u1;
            if (k + 1 < hi) {
                z = -s * en;
                b = c * en;
                x = bn;
            } else {
                e[k * stride] = bn;
                d[(k + 1) * stride] = a_next;
                u[(k + 1) * stride] = u_next;
            }
            a = a_next;
            u0 = u_next;
        }
    }
    return sweeps;
}

}  // namespace slaq
