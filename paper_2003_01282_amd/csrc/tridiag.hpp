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
        // dependent chain of the rotations.  The body has no branch but the
        // rare one for squares out of range (selects instead): a thread
        // running one rotation after another pays no branch per rotation.
        double a = d[lo * stride], b = e[lo * stride], u0 = u[lo * stride];
        double bn = 0.0;
        for (int k = lo; k < hi; ++k) {
            const bool more = k + 1 < hi;
            const double dd = d[(k + 1) * stride];
            const double u1 = u[(k + 1) * stride];
            const double en = more ? e[(k + 1) * stride] : 0.0;
            // rotation with s*x + c*z = 0: the larger of |c|, |s| positive,
            // both from one reciprocal square root of x^2 + z^2 (no division;
            // a ratio-based form guards squares that would over- or underflow)
            double c, s;
            const double r2 = x * x + z * z;
            if (r2 > 1e-290 && r2 < 1e290) {
                const double ri = rsqrt(r2);
                const bool zbig = fabs(z) > fabs(x);
                s = zbig ? fabs(z) * ri : -z * copysign(ri, x);
                c = zbig ? -x * copysign(ri, z) : fabs(x) * ri;
            } else if (fabs(z) > fabs(x)) {
                const double tau = -x / z;
                s = rsqrt(1.0 + tau * tau);
                c = s * tau;
            } else {
                const double tau = -z / x;
                c = rsqrt(1.0 + tau * tau);
                s = c * tau;
            }
            c = z == 0.0 ? 1.0 : c;
            s = z == 0.0 ? 0.0 : s;
            // e[k - 1] is final; at k = lo the store goes to e[lo], which a
            // later rotation or the sweep's end overwrites
            e[(k > lo ? k - 1 : k) * stride] = c * x - s * z;
            const double cc = c * c, ss = s * s, cs = c * s;
            d[k * stride] = a * cc - 2.0 * b * cs + dd * ss;
            const double a_next = a * ss + 2.0 * b * cs + dd * cc;
            bn = (a - dd) * cs + b * (cc - ss);
            u[k * stride] = c * u0 - s * u1;
            const double u_next = s * u0 + c * u1;
            z = more ? -s * en : z;
            b = more ? c * en : b;
            x = more ? bn : x;
            a = a_next;
            u0 = u_next;
        }
        e[(hi - 1) * stride] = bn;
        d[hi * stride] = a;
        u[hi * stride] = u0;
    }
    return sweeps;
}

}  // namespace slaq
