// Host tables of the log-normal coefficient with Hermite chaos (Section 2.1
// and the workload of Section 5).
//
// The coefficient is exp(f) with f the truncated Karhunen-Loeve expansion of
// a Gaussian field with covariance sigma^2 exp(-|x1 - y1| / l - |x2 - y2| / l)
// on [-1, 1]^2 (the unit square of the grid mapped by x = 2 x' - 1), mean
// coefficient 1.  With f_m = sqrt(theta_m) phi_m the Hermite generating
// function gives its chaos coefficients in the orthonormal basis psi_alpha =
// prod He_{alpha_m}(xi_m) / sqrt(alpha_m!):
//   kappa_alpha(x) = prod_m f_m(x)^{alpha_m} / sqrt(alpha_m!),  |alpha| <= 2P,
// n_A = C(M + 2P, 2P) terms.  The operator is sum_l H_l (x) A_l with
// (H_l)_{jk} = E[psi_l psi_j psi_k] = prod_m t(l_m, j_m, k_m), where the 1-D
// product of orthonormal Hermite polynomials is
//   t(a, b, c) = sqrt(a! b! c!) / ((s-a)! (s-b)! (s-c)!),  s = (a+b+c)/2,
// when a + b + c is even and s >= max(a, b, c), and 0 otherwise.
//
// On each element the kernels use B_e = sum_l kappa_l(e) H_l: the Galerkin
// projection E[k_e psi_j psi_k] of the element's coefficient.  Since psi_j
// psi_k has degree <= 2P, the degree-2P truncation projects the exact
// log-normal coefficient, so every B_e is positive definite and so is the SG
// stiffness sum_e B_e (x) K_e.
#include <algorithm>
#include <cmath>

#include "handle.hpp"

namespace sg {

namespace {

double fact(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

// E[psi_a psi_b psi_c], orthonormal probabilists' Hermite polynomials
double hermite_triple(int a, int b, int c) {
    if ((a + b + c) % 2) return 0.0;
    const int s = (a + b + c) / 2;
    if (s < a || s < b || s < c) return 0.0;
    return std::sqrt(fact(a) * fact(b) * fact(c)) / (fact(s - a) * fact(s - b) * fact(s - c));
}

struct KL1 {
    double theta, w, norm;
    int odd;
};

// root of g on (lo, hi) with g(lo), g(hi) of opposite signs, by bisection to
// the last bit
template <typename G>
double bisect(G g, double lo, double hi) {
    double glo = g(lo);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double gm = g(mid);
        if ((gm < 0) == (glo < 0)) {
            lo = mid;
            glo = gm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

// The largest eigenpairs of exp(-|s - t| / corr) on [-1, 1]: theta = 2c / (w^2
// + c^2), c = 1 / corr; even eigenfunctions cos(w x) with c cos(w) - w sin(w) = 0,
// w in (k pi, (k + 1/2) pi); odd ones sin(w x) with w cos(w) + c sin(w) = 0,
// w in ((k + 1/2) pi, (k + 1) pi); normalised on [-1, 1].
std::vector<KL1> kl_1d(int count, double corr) {
    const double c = 1.0 / corr, pi = M_PI, eps = 1e-12;
    std::vector<KL1> out;
    for (int k = 0; (int)out.size() < 2 * count + 2; ++k) {
        double w = bisect([&](double w) { return c * std::cos(w) - w * std::sin(w); }, k * pi + eps,
                          (k + 0.5) * pi - eps);
        out.push_back({2 * c / (w * w + c * c), w, 1.0 / std::sqrt(1.0 + std::sin(2 * w) / (2 * w)), 0});
        w = bisect([&](double w) { return w * std::cos(w) + c * std::sin(w); }, (k + 0.5) * pi + eps,
                   (k + 1) * pi - eps);
        out.push_back({2 * c / (w * w + c * c), w, 1.0 / std::sqrt(1.0 - std::sin(2 * w) / (2 * w)), 1});
    }
    std::stable_sort(out.begin(), out.end(), [](const KL1& a, const KL1& b) { return a.theta > b.theta; });
    out.resize(count);
    return out;
}

double kl_eval(const KL1& p, double x) { return p.norm * (p.odd ? std::sin(p.w * x) : std::cos(p.w * x)); }

}  // namespace

void lognormal_tables(const sg_problem& p, int nxi, const std::vector<int32_t>& alpha, std::vector<double>& H,
                      std::vector<double>& kappa, int& nA) {
    const int M = p.M, P = p.P, n = p.n;
    const std::vector<int32_t> lam = multi_indices(M, 2 * P);
    nA = (int)(lam.size() / M);
    // H_l, dense [l][j][k]
    H.assign((size_t)nA * nxi * nxi, 0.0);
    for (int l = 0; l < nA; ++l)
        for (int j = 0; j < nxi; ++j)
            for (int k = j; k < nxi; ++k) {
                double v = 1.0;
                for (int m = 0; m < M && v != 0.0; ++m)
                    v *= hermite_triple(lam[(size_t)l * M + m], alpha[(size_t)j * M + m], alpha[(size_t)k * M + m]);
                H[((size_t)l * nxi + j) * nxi + k] = H[((size_t)l * nxi + k) * nxi + j] = v;
            }
    // the M largest 2-D eigenpairs: products of 1-D pairs; the unordered
    // index pairs {i <= j} by decreasing eigenvalue, each expanded to (i, j)
    // then (j, i), so that the two equal eigenvalues of a pair keep a fixed
    // order whatever the rounding of the 1-D roots
    const std::vector<KL1> one = kl_1d(M + 2, p.corr_len);
    struct Cand {
        double theta;
        int i, j;
    };
    std::vector<Cand> und, cand;
    for (int i = 0; i < (int)one.size(); ++i)
        for (int j = i; j < (int)one.size(); ++j) und.push_back({p.sigma * p.sigma * one[i].theta * one[j].theta, i, j});
    std::stable_sort(und.begin(), und.end(), [](const Cand& a, const Cand& b) { return a.theta > b.theta; });
    for (const Cand& c : und) {
        cand.push_back(c);
        if (c.i != c.j) cand.push_back({c.theta, c.j, c.i});
    }
    // kappa_l at the element centres, [l][ey][ex]
    kappa.assign((size_t)nA * n * n, 0.0);
    std::vector<double> f(M);
    for (int ey = 0; ey < n; ++ey)
        for (int ex = 0; ex < n; ++ex) {
            const double x1 = 2.0 * (ex + 0.5) / n - 1.0, x2 = 2.0 * (ey + 0.5) / n - 1.0;
            for (int m = 0; m < M; ++m)
                f[m] = std::sqrt(cand[m].theta) * kl_eval(one[cand[m].i], x1) * kl_eval(one[cand[m].j], x2);
            for (int l = 0; l < nA; ++l) {
                double v = 1.0;
                for (int m = 0; m < M; ++m) {
                    const int a = lam[(size_t)l * M + m];
                    if (a) v *= std::pow(f[m], a) / std::sqrt(fact(a));
                }
                kappa[((size_t)l * n + ey) * n + ex] = v;
            }
        }
}

// B_e = sum_{l < r} kappa_l(e) H_l for every element e: [e][j][k]
void lognormal_element_matrices(int n, int nxi, int nA, int r, const std::vector<double>& H,
                                const std::vector<double>& kappa, double* B) {
    const size_t ne = (size_t)n * n, nn = (size_t)nxi * nxi;
    // the nonzero entries of each H_l once
    std::vector<std::vector<std::pair<int, double>>> nz(r);
    for (int l = 0; l < r && l < nA; ++l)
        for (size_t q = 0; q < nn; ++q)
            if (H[l * nn + q] != 0.0) nz[l].push_back({(int)q, H[l * nn + q]});
    for (size_t e = 0; e < ne; ++e) {
        double* b = B + e * nn;
        std::fill(b, b + nn, 0.0);
        for (int l = 0; l < r && l < nA; ++l) {
            const double k = kappa[l * ne + e];
            for (const auto& q : nz[l]) b[q.first] += k * q.second;
        }
    }
}

}  // namespace sg
