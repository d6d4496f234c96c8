// Host-side spectral helpers for the polynomial preconditioner (Section 4.7).
//
// hessenberg_eigvals: eigenvalues of a small upper Hessenberg matrix by the
// implicitly double-shifted QR iteration (Francis step with 3x3 Householder
// bulge chasing and deflation on negligible subdiagonals; Golub & Van Loan,
// Matrix Computations, Section 7.5). Only the active diagonal window is
// transformed since no eigenvectors are needed.
//
// harmonic_ritz_leja: harmonic Ritz values from one Arnoldi cycle, i.e. the
// eigenvalues of H_P + h_{P+1,P}^2 H_P^{-T} e_P e_P^T, then a Leja ordering
// (first the value of largest modulus, then repeatedly the candidate that
// maximises the product of distances to the values already chosen) with each
// complex value immediately followed by its conjugate.
// poly_roots: the same values plus the safeguard's added copy of the outermost root.
#include <cfloat>
#include <cmath>
#include <vector>

#include "hdg_internal.hpp"

namespace {

void house(int n, const double* a, double* v, double* beta) {
    // v such that (I - beta v v^T) a = alpha e1
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) {
        *beta = 0.0;
        for (int i = 0; i < n; ++i) v[i] = 0.0;
        return;
    }
    const double alpha = a[0] >= 0.0 ? -nrm : nrm;
    v[0] = a[0] - alpha;
    for (int i = 1; i < n; ++i) v[i] = a[i];
    double vv = 0.0;
    for (int i = 0; i < n; ++i) vv += v[i] * v[i];
    *beta = vv > 0.0 ? 2.0 / vv : 0.0;
}

}  // namespace

int hessenberg_eigvals(int n, double* H, int ld, double* wr, double* wi) {
    auto h = [&](int i, int j) -> double& { return H[(size_t)i * ld + j]; };
    double anorm = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) anorm += std::fabs(h(i, j));
    if (anorm == 0.0) anorm = 1.0;
    int hi = n - 1;
    int iter = 0, total = 0;
    while (hi >= 0) {
        int lo = hi;
        while (lo > 0) {
            double s = std::fabs(h(lo - 1, lo - 1)) + std::fabs(h(lo, lo));
            if (s == 0.0) s = anorm;
            if (std::fabs(h(lo, lo - 1)) <= DBL_EPSILON * s) {
                h(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            wr[hi] = h(hi, hi);
            wi[hi] = 0.0;
            --hi;
            iter = 0;
            continue;
        }
        if (lo == hi - 1) {
            const double a = h(lo, lo), b = h(lo, hi), c = h(hi, lo), d = h(hi, hi);
            const double mid = 0.5 * (a + d);
            const double disc = 0.25 * (a - d) * (a - d) + b * c;
            if (disc >= 0.0) {
                const double sq = std::sqrt(disc);
                const double r1 = mid + (mid >= 0.0 ? sq : -sq);
                const double det = a * d - b * c;
                const double r2 = r1 != 0.0 ? det / r1 : mid - sq;
                wr[lo] = r1; wi[lo] = 0.0;
                wr[hi] = r2; wi[hi] = 0.0;
            } else {
                const double im = std::sqrt(-disc);
                wr[lo] = mid; wi[lo] = im;
                wr[hi] = mid; wi[hi] = -im;
            }
            hi -= 2;
            iter = 0;
            continue;
        }
        ++iter;
        if (++total > 200 * n) return -1;
        double s, t;
        if (iter % 11 == 10) {
            const double ex = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
            s = 1.5 * ex;
            t = ex * ex;
        } else {
            s = h(hi - 1, hi - 1) + h(hi, hi);
            t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
        }
        double a3[3];
        a3[0] = h(lo, lo) * h(lo, lo) + h(lo, lo + 1) * h(lo + 1, lo) - s * h(lo, lo) + t;
        a3[1] = h(lo + 1, lo) * (h(lo, lo) + h(lo + 1, lo + 1) - s);
        a3[2] = h(lo + 1, lo) * h(lo + 2, lo + 1);
        for (int k = lo; k <= hi - 2; ++k) {
            double v[3], beta;
            house(3, a3, v, &beta);
            if (beta != 0.0) {
                const int c0 = k - 1 > lo ? k - 1 : lo;
                for (int j = c0; j <= hi; ++j) {
                    const double dot = v[0] * h(k, j) + v[1] * h(k + 1, j) + v[2] * h(k + 2, j);
                    h(k, j) -= beta * v[0] * dot;
                    h(k + 1, j) -= beta * v[1] * dot;
                    h(k + 2, j) -= beta * v[2] * dot;
                }
                const int r1 = k + 3 < hi ? k + 3 : hi;
                for (int i = lo; i <= r1; ++i) {
                    const double dot = h(i, k) * v[0] + h(i, k + 1) * v[1] + h(i, k + 2) * v[2];
                    h(i, k) -= beta * dot * v[0];
                    h(i, k + 1) -= beta * dot * v[1];
                    h(i, k + 2) -= beta * dot * v[2];
                }
            }
            a3[0] = h(k + 1, k);
            a3[1] = h(k + 2, k);
            a3[2] = (k < hi - 2) ? h(k + 3, k) : 0.0;
        }
        double v[2], beta;
        house(2, a3, v, &beta);
        if (beta != 0.0) {
            const int c0 = hi - 2 > lo ? hi - 2 : lo;
            for (int j = c0; j <= hi; ++j) {
                const double dot = v[0] * h(hi - 1, j) + v[1] * h(hi, j);
                h(hi - 1, j) -= beta * v[0] * dot;
                h(hi, j) -= beta * v[1] * dot;
            }
            for (int i = lo; i <= hi; ++i) {
                const double dot = h(i, hi - 1) * v[0] + h(i, hi) * v[1];
                h(i, hi - 1) -= beta * dot * v[0];
                h(i, hi) -= beta * dot * v[1];
            }
        }
    }
    return 0;
}

namespace {

// Harmonic Ritz values of one Arnoldi cycle: the eigenvalues of H_P + h^2 f e_P^T with
// H_P^T f = e_P (H is (P+1) x P, row-major).
int harmonic_values(int P, const double* H, std::vector<double>& wr, std::vector<double>& wi) {
    std::vector<double> Hm((size_t)P * P), At((size_t)P * P), f(P, 0.0);
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            Hm[(size_t)i * P + j] = H[(size_t)i * P + j];
            At[(size_t)i * P + j] = H[(size_t)j * P + i];   // transpose
        }
    const double hs = H[(size_t)P * P + (P - 1)];
    f[P - 1] = 1.0;
    // Gaussian elimination with partial pivoting on At f = e_P
    bool ok = true;
    for (int k = 0; k < P && ok; ++k) {
        int p = k;
        for (int i = k + 1; i < P; ++i)
            if (std::fabs(At[(size_t)i * P + k]) > std::fabs(At[(size_t)p * P + k])) p = i;
        if (At[(size_t)p * P + k] == 0.0) { ok = false; break; }
        if (p != k) {
            for (int j = 0; j < P; ++j) std::swap(At[(size_t)k * P + j], At[(size_t)p * P + j]);
            std::swap(f[k], f[p]);
        }
        for (int i = k + 1; i < P; ++i) {
            const double m = At[(size_t)i * P + k] / At[(size_t)k * P + k];
            for (int j = k; j < P; ++j) At[(size_t)i * P + j] -= m * At[(size_t)k * P + j];
            f[i] -= m * f[k];
        }
    }
    if (ok) {
        for (int i = P - 1; i >= 0; --i) {
            double s = f[i];
            for (int j = i + 1; j < P; ++j) s -= At[(size_t)i * P + j] * f[j];
            f[i] = s / At[(size_t)i * P + i];
        }
        for (int i = 0; i < P; ++i) Hm[(size_t)i * P + (P - 1)] += hs * hs * f[i];
    }
    wr.assign(P, 0.0);
    wi.assign(P, 0.0);
    return hessenberg_eigvals(P, Hm.data(), P, wr.data(), wi.data()) != 0 ? -2 : 0;
}

// Leja order of the candidates (real values and the positive-imaginary member of each pair):
// first the largest modulus, then repeatedly the candidate maximising the sum of log distances
// to the values already chosen (a candidate equal to a chosen value scores minus infinity; ties
// to the lower index); each complex value is followed by its conjugate.
void leja(const std::vector<double>& cr, const std::vector<double>& ci, double* tre, double* tim, int* nout) {
    const int nc = (int)cr.size();
    std::vector<char> used(nc, 0);
    std::vector<double> sr, si;   // selected values (both members of pairs)
    for (int step = 0; step < nc; ++step) {
        int best = -1;
        double bscore = -INFINITY;
        for (int c = 0; c < nc; ++c) {
            if (used[c]) continue;
            double score;
            if (sr.empty()) {
                score = std::hypot(cr[c], ci[c]);
            } else {
                score = 0.0;
                for (size_t q = 0; q < sr.size(); ++q) {
                    const double dist = std::hypot(cr[c] - sr[q], ci[c] - si[q]);
                    score += dist > 0.0 ? std::log(dist) : -INFINITY;
                }
            }
            if (best < 0 || score > bscore) { best = c; bscore = score; }
        }
        used[best] = 1;
        tre[*nout] = cr[best];
        tim[*nout] = ci[best];
        ++*nout;
        sr.push_back(cr[best]);
        si.push_back(ci[best]);
        if (ci[best] > 0.0) {
            tre[*nout] = cr[best];
            tim[*nout] = -ci[best];
            ++*nout;
            sr.push_back(cr[best]);
            si.push_back(-ci[best]);
        }
    }
}

// The candidates of the harmonic Ritz values whose modulus is at least drop_rel of the largest.
void candidates(const std::vector<double>& wr, const std::vector<double>& wi, double drop_rel,
                std::vector<double>& cr, std::vector<double>& ci) {
    double amax = 0.0;
    for (size_t i = 0; i < wr.size(); ++i) amax = std::fmax(amax, std::hypot(wr[i], wi[i]));
    for (size_t i = 0; i < wr.size(); ++i) {
        if (std::hypot(wr[i], wi[i]) < drop_rel * amax) continue;
        if (wi[i] < 0.0) continue;
        cr.push_back(wr[i]);
        ci.push_back(wi[i]);
    }
}

}  // namespace

int harmonic_ritz_leja(int P, const double* H, double drop_rel, double* tre, double* tim, int* nout) {
    *nout = 0;
    if (P < 1) return -1;
    std::vector<double> wr, wi, cr, ci;
    if (harmonic_values(P, H, wr, wi) != 0) return -2;
    candidates(wr, wi, drop_rel, cr, ci);
    leja(cr, ci, tre, tim, nout);
    return 0;
}

// The roots the polynomial preconditioner uses: the harmonic Ritz values (small ones dropped)
// plus, as a safeguard, up to two more copies of the root of largest real part t (and of its
// conjugate), each added while the residual polynomial pi(z) = prod_j (1 - z/theta_j) has
// modulus above 1 at 1.1 t -- the spectrum of B can reach beyond the outermost harmonic Ritz
// value, and there 1 - pi(z) = z p(z) turns negative -- all in Leja order. tre/tim need P + 4
// entries.
int poly_roots(int P, const double* H, double drop_rel, double* tre, double* tim, int* nout, int* nadded) {
    *nout = 0;
    *nadded = 0;
    if (P < 1) return -1;
    std::vector<double> wr, wi, cr, ci;
    if (harmonic_values(P, H, wr, wi) != 0) return -2;
    candidates(wr, wi, drop_rel, cr, ci);
    int nval = 0;
    for (size_t c = 0; c < cr.size(); ++c) nval += ci[c] > 0.0 ? 2 : 1;
    if (nval >= 2) {
        size_t k = 0;
        for (size_t c = 1; c < cr.size(); ++c)
            if (cr[c] > cr[k]) k = c;
        const double tr = cr[k], ti = ci[k];
        // at most two more copies, each added while |pi(1.1 t)| > 1 over every value (both
        // members of the pairs, the copies included)
        for (int copy = 0; copy < 2 && tr > 0.0; ++copy) {
            const double zr = 1.1 * tr, zi = 1.1 * ti;
            double pr = 1.0, pim = 0.0;
            for (size_t c = 0; c < cr.size(); ++c) {
                for (int sgn = 1; sgn >= (ci[c] > 0.0 ? -1 : 1); sgn -= 2) {
                    const double a = cr[c], b = sgn * ci[c];
                    const double den = a * a + b * b;
                    // 1 - z / theta = 1 - z conj(theta) / |theta|^2
                    const double fr = 1.0 - (zr * a + zi * b) / den;
                    const double fi = -(zi * a - zr * b) / den;
                    const double nr = pr * fr - pim * fi;
                    pim = pr * fi + pim * fr;
                    pr = nr;
                }
            }
            if (!(std::hypot(pr, pim) > 1.0)) break;
            cr.push_back(tr);
            ci.push_back(ti);
            *nadded += ti > 0.0 ? 2 : 1;
        }
    }
    leja(cr, ci, tre, tim, nout);
    return 0;
}
