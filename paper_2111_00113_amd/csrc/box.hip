// Spectral box for the Chebyshev basis from a short Arnoldi pass
// (arXiv:2111.00113 Section 4.4: estimate the spectrum with a few Arnoldi
// iterations, then fit the Chebyshev polynomials to a region containing it).
//
// Host code: the m x m Hessenberg matrix of an m-step Arnoldi process (built
// on the GPU by the resident basis kernel with a full window) has the Ritz
// values as eigenvalues; they are computed here by the implicitly
// double-shifted QR iteration, and the box [c +- dx] x [+-dy] is their
// bounding rectangle widened by a fixed margin.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace sg {

namespace {

// Householder reflector for (x0, ..., x_{len-1}) (len 2 or 3): v and
// beta = 2 / v^T v with (I - beta v v^T) x = (alpha, 0, ...), alpha =
// -sign(x0) |x|.  beta = 0 when x = 0 (identity).
void reflector(int len, const double* x, double* v, double* beta, double* alpha) {
    double nrm = 0.0;
    for (int i = 0; i < len; ++i) nrm = std::hypot(nrm, x[i]);
    if (nrm == 0.0) {
        for (int i = 0; i < len; ++i) v[i] = 0.0;
        *beta = 0.0;
        *alpha = 0.0;
        return;
    }
    const double a = x[0] >= 0.0 ? -nrm : nrm;
    v[0] = x[0] - a;
    for (int i = 1; i < len; ++i) v[i] = x[i];
    double vtv = 0.0;
    for (int i = 0; i < len; ++i) vtv += v[i] * v[i];
    *beta = 2.0 / vtv;
    *alpha = a;
}

}  // namespace

// Eigenvalues of the m x m upper Hessenberg matrix H (column-major, leading
// dimension ldh; entries below the subdiagonal are ignored; H is overwritten)
// by Francis double-shift QR steps on the trailing unreduced block, deflating
// at subdiagonal entries below eps (|h_{i-1,i-1}| + |h_{ii}|).  Returns 0, or
// -1 when a block has not split after 100 steps.
int hessenberg_eigenvalues(int m, double* Hm, int ldh, double* wr, double* wi) {
    auto H = [&](int i, int j) -> double& { return Hm[i + static_cast<int64_t>(j) * ldh]; };
    const double eps = 0x1.0p-52;
    double anorm = 0.0;
    for (int j = 0; j < m; ++j)
        for (int i = 0; i <= std::min(j + 1, m - 1); ++i) anorm = std::max(anorm, std::fabs(H(i, j)));
    int hi = m - 1;
    int iter = 0;
    while (hi >= 0) {
        // the active block is [l, hi]: l is the first row below a negligible
        // subdiagonal entry
        int l = hi;
        while (l > 0) {
            double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
            if (s == 0.0) s = anorm;
            if (std::fabs(H(l, l - 1)) <= eps * s) {
                H(l, l - 1) = 0.0;
                break;
            }
            --l;
        }
        if (l == hi) {  // a 1 x 1 block
            wr[hi] = H(hi, hi);
            wi[hi] = 0.0;
            --hi;
            iter = 0;
            continue;
        }
        if (l == hi - 1) {  // a 2 x 2 block: its eigenvalues in closed form
            const double a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
            const double p = 0.5 * (a - d);
            const double disc = p * p + b * c;
            if (disc >= 0.0) {
                const double z = p + std::copysign(std::sqrt(disc), p);
                wr[hi - 1] = d + z;
                wr[hi] = z != 0.0 ? d - b * c / z : d;
                wi[hi - 1] = wi[hi] = 0.0;
            } else {
                wr[hi - 1] = wr[hi] = d + p;
                wi[hi - 1] = std::sqrt(-disc);
                wi[hi] = -wi[hi - 1];
            }
            hi -= 2;
            iter = 0;
            continue;
        }
        if (++iter > 100) return -1;
        // shifts: the eigenvalues of the trailing 2 x 2 block (sum s,
        // product t), replaced by ad hoc ones every tenth step
        double s = H(hi - 1, hi - 1) + H(hi, hi);
        double t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
        if (iter % 10 == 0) {
            const double w = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
            s = 1.5 * w;
            t = w * w;
        }
        // first column of (H - s1 I)(H - s2 I) = H^2 - s H + t I
        double x[3] = {H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t,
                       H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s), H(l + 1, l) * H(l + 2, l + 1)};
        // chase the bulge down the active block
        for (int k = l; k <= hi - 1; ++k) {
            const int len = k <= hi - 2 ? 3 : 2;
            double v[3], beta, alpha;
            reflector(len, x, v, &beta, &alpha);
            if (k > l) {
                H(k, k - 1) = alpha;
                for (int i = 1; i < len; ++i) H(k + i, k - 1) = 0.0;
            }
            if (beta != 0.0) {
                for (int j = k; j <= hi; ++j) {  // from the left: rows k .. k + len - 1
                    double dot = 0.0;
                    for (int i = 0; i < len; ++i) dot += v[i] * H(k + i, j);
                    const double f = beta * dot;
                    for (int i = 0; i < len; ++i) H(k + i, j) -= f * v[i];
                }
                const int rmax = std::min(k + 3, hi);
                for (int r = l; r <= rmax; ++r) {  // from the right: columns k .. k + len - 1
                    double dot = 0.0;
                    for (int i = 0; i < len; ++i) dot += H(r, k + i) * v[i];
                    const double f = beta * dot;
                    for (int i = 0; i < len; ++i) H(r, k + i) -= f * v[i];
                }
            }
            if (k < hi - 1) {
                x[0] = H(k + 1, k);
                x[1] = H(k + 2, k);
                x[2] = k < hi - 2 ? H(k + 3, k) : 0.0;
            }
        }
    }
    return 0;
}

void box_from_ritz(int m, const double* wr, const double* wi, double margin, double box[3]) {
    double xmin = wr[0], xmax = wr[0], ymax = 0.0;
    for (int i = 0; i < m; ++i) {
        xmin = std::min(xmin, wr[i]);
        xmax = std::max(xmax, wr[i]);
        ymax = std::max(ymax, std::fabs(wi[i]));
    }
    box[0] = 0.5 * (xmin + xmax);
    box[1] = (1.0 + margin) * 0.5 * (xmax - xmin);
    box[2] = (1.0 + margin) * ymax;
}

}  // namespace sg
