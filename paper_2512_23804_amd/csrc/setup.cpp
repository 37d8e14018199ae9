// Host-side setup: validation, multi-index set, triple-product neighbour
// table, per-element coefficient modes, multigrid constants, right-hand sides,
// and the upload of all of it to the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "handle.hpp"

namespace sg {

int binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int)r;
}

void default_options(sg_options* o) {
    o->rtol = 1e-8;
    o->restart = 30;
    o->max_iter = 600;
    o->cheb_steps = 5;
    o->truncation_r = 0;
    o->gmg_pre = 2;
    o->gmg_post = 2;
    o->precision = SG_PREC_FP64;
    o->inner_rtol = 1e-5;
    o->use_graphs = 1;
    o->verbose = 0;
    o->profile = SG_PROF_NONE;
    o->arnoldi = SG_ARNOLDI_DCGS2;
    o->sweep_rows = 0;
    o->basis_fp32 = 1;
    o->mean_solver = SG_MEAN_MULTIGRID;
    o->richardson_steps = 1;
    o->precond = SG_PRECOND_BLOCK_DIAGONAL;
}

// Total-degree multi-indices, degree ascending, descending lexicographic order
// inside a degree (Section 2.1 dimension C(M+P, P); Algorithm 1 level ranges).
static void compositions(int total, int parts, std::vector<int>& cur, std::vector<int32_t>& out) {
    if (parts == 1) {
        cur.push_back(total);
        out.insert(out.end(), cur.begin(), cur.end());
        cur.pop_back();
        return;
    }
    for (int first = total; first >= 0; --first) {
        cur.push_back(first);
        compositions(total - first, parts - 1, cur, out);
        cur.pop_back();
    }
}

std::vector<int32_t> multi_indices(int M, int P) {
    std::vector<int32_t> out;
    std::vector<int> cur;
    for (int d = 0; d <= P; ++d) compositions(d, M, cur, out);
    return out;
}

static bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

static void fail(int code, const std::string& m) { throw Error(code, m); }

// Per-element coefficient modes of one problem: [M+1][n][n].
static std::vector<double> coefficient_modes(const sg_problem& p) {
    const int n = p.n, M = p.M;
    std::vector<double> c((size_t)(M + 1) * n * n);
    if (p.field == SG_FIELD_LOGNORMAL) {
        // the mean coefficient (kappa_1 = 1); the log-normal terms live in the
        // element couplings of the general kernels
        std::fill(c.begin(), c.begin() + (size_t)n * n, 1.0);
        return c;
    }
    if (p.kappa) {
        std::memcpy(c.data(), p.kappa, c.size() * sizeof(double));
        return c;
    }
    // a = 1 + sigma sum_k k^-2 cos(k pi x1) cos(k pi x2) xi_k; xi_k = psi_{e_k}/sqrt(3)
    const double h = 1.0 / n;
    for (int ey = 0; ey < n; ++ey)
        for (int ex = 0; ex < n; ++ex) c[(size_t)ey * n + ex] = 1.0;
    for (int k = 1; k <= M; ++k) {
        const double amp = p.sigma / ((double)k * k) / std::sqrt(3.0);
        for (int ey = 0; ey < n; ++ey) {
            const double cy = std::cos(k * M_PI * (ey + 0.5) * h);
            for (int ex = 0; ex < n; ++ex)
                c[((size_t)k * n + ey) * n + ex] = amp * std::cos(k * M_PI * (ex + 0.5) * h) * cy;
        }
    }
    return c;
}

void validate(const sg_problem* probs, int count, const sg_options* opt) {
    if (!probs || count < 1) fail(SG_ERR_INVALID, "no problems given");
    if (count > 2048) fail(SG_ERR_INVALID, "too many members in one batch (max 2048)");
    const sg_problem& p0 = probs[0];
    for (int i = 0; i < count; ++i) {
        const sg_problem& p = probs[i];
        const std::string who = "problem " + std::to_string(i) + ": ";
        if (!is_pow2(p.n) || p.n < 8 || p.n > 4096) fail(SG_ERR_INVALID, who + "n must be a power of two in [8, 4096]");
        if (p.M < 1 || p.M > kMaxM) fail(SG_ERR_INVALID, who + "M must be in [1, 16]");
        if (p.P < 1 || p.P > kMaxP) fail(SG_ERR_INVALID, who + "P must be in [1, 8]");
        if (binom(p.M + p.P, p.P) > 20000) fail(SG_ERR_INVALID, who + "chaos dimension above 20000");
        if (p.n_t > 4096) fail(SG_ERR_INVALID, who + "n_t above 4096");
        if (p.n != p0.n || p.M != p0.M || p.P != p0.P || std::max(p.n_t, 1) != std::max(p0.n_t, 1))
            fail(SG_ERR_INVALID, who + "members of one batch must share n, M, P, n_t");
        if (p.field != SG_FIELD_AFFINE && p.field != SG_FIELD_LOGNORMAL)
            fail(SG_ERR_INVALID, who + "field must be SG_FIELD_AFFINE or SG_FIELD_LOGNORMAL");
        if (p.field != p0.field) fail(SG_ERR_INVALID, who + "members of one batch must share the field model");
        if (!std::isfinite(p.beta) || !std::isfinite(p.gamma) || !std::isfinite(p.sigma) ||
            (p.n_t >= 2 && !std::isfinite(p.T)))
            fail(SG_ERR_NONFINITE, who + "non-finite scalar parameter");
        if (!(p.beta > 0)) fail(SG_ERR_INVALID, who + "beta must be > 0");
        if (!(p.gamma >= 0)) fail(SG_ERR_INVALID, who + "gamma must be >= 0");
        if (p.n_t >= 2 && !(p.T > 0)) fail(SG_ERR_INVALID, who + "T must be > 0");
        if (!p.kappa && !(p.sigma >= 0)) fail(SG_ERR_INVALID, who + "sigma must be >= 0");
        if (!p.y_target) fail(SG_ERR_INVALID, who + "y_target is NULL");
        const int nt = std::max(p.n_t, 1);
        const size_t nodes = (size_t)(p.n + 1) * (p.n + 1);
        for (size_t q = 0; q < nt * nodes; ++q)
            if (!std::isfinite(p.y_target[q])) fail(SG_ERR_NONFINITE, who + "non-finite target value");
        if (p.y0) {
            if (p.n_t < 2) fail(SG_ERR_INVALID, who + "y0 given for a steady problem");
            for (size_t q = 0; q < nodes; ++q)
                if (!std::isfinite(p.y0[q])) fail(SG_ERR_NONFINITE, who + "non-finite initial state");
        }
        if (p.field == SG_FIELD_LOGNORMAL) {
            // exp of a Gaussian field: positive for every xi, and its degree-2P chaos
            // projection gives positive definite element couplings (lognormal.cpp)
            if (p.kappa) fail(SG_ERR_INVALID, who + "kappa must be NULL for the log-normal field");
            if (!std::isfinite(p.corr_len) || !(p.corr_len > 0)) fail(SG_ERR_INVALID, who + "corr_len must be > 0");
            if (!(p.sigma >= 0)) fail(SG_ERR_INVALID, who + "sigma must be >= 0");
            const double nxi = binom(p.M + p.P, p.P);
            if (nxi > 256) fail(SG_ERR_INVALID, who + "log-normal field: chaos dimension above 256");
            if ((double)p.n * p.n * nxi * nxi * 8.0 > 8.0 * (1ull << 30))
                fail(SG_ERR_INVALID, who + "log-normal field: element coupling tables above 8 GiB per member");
            continue;
        }
        // coefficient: finite, constant positive mean, bounded away from zero for all xi
        const size_t ne = (size_t)p.n * p.n;
        if (p.kappa) {
            for (size_t q = 0; q < (size_t)(p.M + 1) * ne; ++q)
                if (!std::isfinite(p.kappa[q])) fail(SG_ERR_NONFINITE, who + "non-finite coefficient mode");
            for (size_t q = 1; q < ne; ++q)
                if (p.kappa[q] != p.kappa[0]) fail(SG_ERR_INVALID, who + "kappa_0 must be constant");
        }
        const double c0 = p.kappa ? p.kappa[0] : 1.0;
        if (!(c0 > 0)) fail(SG_ERR_NONCOERCIVE, who + "mean coefficient must be positive");
        double worst = INFINITY;
        if (p.kappa) {
            for (size_t e = 0; e < ne; ++e) {
                double s = 0.0;
                for (int k = 1; k <= p.M; ++k) s += std::fabs(p.kappa[(size_t)k * ne + e]);
                worst = std::min(worst, c0 - std::sqrt(3.0) * s);
            }
        } else {
            const double h = 1.0 / p.n;
            for (int ey = 0; ey < p.n; ++ey)
                for (int ex = 0; ex < p.n; ++ex) {
                    double s = 0.0;
                    for (int k = 1; k <= p.M; ++k)
                        s += std::fabs(std::cos(k * M_PI * (ex + 0.5) * h) * std::cos(k * M_PI * (ey + 0.5) * h)) /
                             ((double)k * k);
                    worst = std::min(worst, 1.0 - p.sigma * s);
                }
        }
        if (!(worst > 0)) fail(SG_ERR_NONCOERCIVE, who + "coefficient is not bounded away from zero for xi in [-1,1]^M");
    }
    if (opt) {
        if (!(opt->rtol > 0) || !std::isfinite(opt->rtol)) fail(SG_ERR_INVALID, "rtol must be > 0");
        if (opt->restart < 1 || opt->restart > 31) fail(SG_ERR_INVALID, "restart must be in [1, 31]");
        if (opt->max_iter < 1) fail(SG_ERR_INVALID, "max_iter must be >= 1");
        if (opt->cheb_steps < 0 || opt->cheb_steps > 64)
            fail(SG_ERR_INVALID, "cheb_steps must be in [0, 64] (0: exact mass solves)");
        if (opt->mean_solver != SG_MEAN_MULTIGRID && opt->mean_solver != SG_MEAN_EXACT)
            fail(SG_ERR_INVALID, "mean_solver must be SG_MEAN_MULTIGRID or SG_MEAN_EXACT");
        if (opt->richardson_steps < 1 || opt->richardson_steps > 16)
            fail(SG_ERR_INVALID, "richardson_steps must be in [1, 16]");
        if (opt->precond != SG_PRECOND_BLOCK_DIAGONAL && opt->precond != SG_PRECOND_HGSOC)
            fail(SG_ERR_INVALID, "precond must be SG_PRECOND_BLOCK_DIAGONAL or SG_PRECOND_HGSOC");
        if (opt->precond == SG_PRECOND_HGSOC && (opt->cheb_steps < 1 || opt->cheb_steps > 9))
            fail(SG_ERR_INVALID, "hGSoc needs cheb_steps in [1, 9]");
        const int nterms = p0.field == SG_FIELD_LOGNORMAL ? binom(p0.M + 2 * p0.P, 2 * p0.P) : p0.M + 1;
        if (opt->truncation_r < 0 || opt->truncation_r > nterms)
            fail(SG_ERR_INVALID, "truncation_r must be in [0, number of coefficient terms] (M+1 affine, "
                                 "C(M+2P, 2P) log-normal)");
        if (opt->gmg_pre < 1 || opt->gmg_pre > kMaxSmooth || opt->gmg_post < 1 || opt->gmg_post > kMaxSmooth)
            fail(SG_ERR_INVALID, "gmg_pre/gmg_post must be in [1, 4]");
        if (opt->precision != SG_PREC_FP64 && opt->precision != SG_PREC_FP32_REFINE &&
            opt->precision != SG_PREC_FP32_PRECOND)
            fail(SG_ERR_INVALID, "unknown precision mode");
        if (opt->profile < SG_PROF_NONE || opt->profile > SG_PROF_MG_UP) fail(SG_ERR_INVALID, "unknown profile kind");
        if (opt->sweep_rows != 0 && opt->sweep_rows != 2 && opt->sweep_rows != 4 && opt->sweep_rows != 8)
            fail(SG_ERR_INVALID, "sweep_rows must be 0 (autotune), 2, 4 or 8");
        if (opt->basis_fp32 != 0 && opt->basis_fp32 != 1) fail(SG_ERR_INVALID, "basis_fp32 must be 0 or 1");
        if (opt->arnoldi != SG_ARNOLDI_DCGS2 && opt->arnoldi != SG_ARNOLDI_CGS2)
            fail(SG_ERR_INVALID, "arnoldi must be SG_ARNOLDI_DCGS2 or SG_ARNOLDI_CGS2");
        if (opt->precision == SG_PREC_FP32_REFINE && !(opt->inner_rtol > 0 && opt->inner_rtol < 1))
            fail(SG_ERR_INVALID, "inner_rtol must be in (0, 1)");
    }
}

// Largest eigenvalue of diag(A)^{-1} A for A = a K + b M_h on the interior of
// the m x m grid: the Q1 matrices are Kronecker sums of 1-D P1 matrices whose
// common eigenvectors are discrete sines (1-D eigenvalues (2/h)(1 - cos t) for
// the stiffness and (h/3)(2 + cos t) for the mass, t = i pi h).
static double lambda_max(int m, double a, double b) {
    const double h = 1.0 / m;
    std::vector<double> k1(m - 1), m1(m - 1);
    for (int i = 1; i < m; ++i) {
        const double t = i * M_PI * h;
        k1[i - 1] = (2.0 / h) * (1.0 - std::cos(t));
        m1[i - 1] = (h / 3.0) * (2.0 + std::cos(t));
    }
    double best = 0.0;
    for (int i = 0; i < m - 1; ++i)
        for (int j = 0; j < m - 1; ++j) {
            const double lam = a * (k1[i] * m1[j] + m1[i] * k1[j]) + b * m1[i] * m1[j];
            best = std::max(best, lam);
        }
    const double diag = a * 8.0 / 3.0 + b * 4.0 * h * h / 9.0;
    return best / diag;
}

// Chebyshev smoothing coefficients on [0.3, 1.1] * lambda_max of D^{-1} A:
// step 0: d = D^{-1} r / theta; step i: rho_i = 1/(2 sigma - rho_{i-1}),
// d = rho_i rho_{i-1} d + (2 rho_i / delta) D^{-1} r.
static void smoother_coeffs(double lmax, int nu, double out[kMaxSmooth][2]) {
    const double lo = 0.3 * lmax, hi = 1.1 * lmax;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    const double sig = theta / delta;
    double rho_old = 1.0 / sig;
    for (int s = 0; s < kMaxSmooth; ++s) out[s][0] = out[s][1] = 0.0;
    out[0][0] = 0.0;
    out[0][1] = 1.0 / theta;
    for (int s = 1; s < nu; ++s) {
        const double rho = 1.0 / (2.0 * sig - rho_old);
        out[s][0] = rho * rho_old;
        out[s][1] = 2.0 * rho / delta;
        rho_old = rho;
    }
}

// Inverse of a K + b M on the interior of the kCoarseN grid, padded to 64 x 64.
static void coarse_inverse(double a, double b, double* out) {
    const int m = kCoarseN, nu = (m - 1) * (m - 1);
    const double h = 1.0 / m;
    std::vector<double> A((size_t)nu * nu, 0.0), I((size_t)nu * nu, 0.0);
    const double wc = a * 8.0 / 3.0 + b * 16.0 * h * h / 36.0;
    const double we = -a / 3.0 + b * 4.0 * h * h / 36.0;
    const double wd = -a / 3.0 + b * h * h / 36.0;
    for (int iy = 1; iy < m; ++iy)
        for (int ix = 1; ix < m; ++ix) {
            const int r = (iy - 1) * (m - 1) + (ix - 1);
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int jx = ix + dx, jy = iy + dy;
                    if (jx < 1 || jx > m - 1 || jy < 1 || jy > m - 1) continue;
                    const int c = (jy - 1) * (m - 1) + (jx - 1);
                    const double w = (dx == 0 && dy == 0) ? wc : (dx == 0 || dy == 0) ? we : wd;
                    A[(size_t)r * nu + c] = w;
                }
            I[(size_t)r * nu + r] = 1.0;
        }
    // Gauss-Jordan elimination with partial pivoting
    for (int col = 0; col < nu; ++col) {
        int piv = col;
        for (int r = col + 1; r < nu; ++r)
            if (std::fabs(A[(size_t)r * nu + col]) > std::fabs(A[(size_t)piv * nu + col])) piv = r;
        if (piv != col)
            for (int c = 0; c < nu; ++c) {
                std::swap(A[(size_t)piv * nu + c], A[(size_t)col * nu + c]);
                std::swap(I[(size_t)piv * nu + c], I[(size_t)col * nu + c]);
            }
        const double d = A[(size_t)col * nu + col];
        for (int c = 0; c < nu; ++c) {
            A[(size_t)col * nu + c] /= d;
            I[(size_t)col * nu + c] /= d;
        }
        for (int r = 0; r < nu; ++r) {
            if (r == col) continue;
            const double f = A[(size_t)r * nu + col];
            if (f == 0.0) continue;
            for (int c = 0; c < nu; ++c) {
                A[(size_t)r * nu + c] -= f * A[(size_t)col * nu + c];
                I[(size_t)r * nu + c] -= f * I[(size_t)col * nu + c];
            }
        }
    }
    std::fill(out, out + kCoarsePad * kCoarsePad, 0.0);
    for (int r = 0; r < nu; ++r)
        for (int c = 0; c < nu; ++c) out[r * kCoarsePad + c] = I[(size_t)r * nu + c];
}

// Pinned host staging buffers (4096 doubles) are kept for reuse: the server
// builds a handle per batch, and pinned allocations are slow.
namespace {
std::mutex g_pinned_mu;
std::vector<double*> g_pinned_free;
}  // namespace

static double* pinned_get() {
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        if (!g_pinned_free.empty()) {
            double* p = g_pinned_free.back();
            g_pinned_free.pop_back();
            return p;
        }
    }
    double* p = nullptr;
    SG_HIP(hipHostMalloc((void**)&p, kPinnedDoubles * sizeof(double), hipHostMallocDefault));
    return p;
}

static void pinned_put(double* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    if (g_pinned_free.size() < 64)
        g_pinned_free.push_back(p);
    else
        (void)hipHostFree(p);
}

Handle::~Handle() {
    ws.release();
    for (void* p : {(void*)d_nbr_idx, (void*)d_nbr_val, (void*)d_coef64, (void*)d_coef32, (void*)d_mem,
                    (void*)d_lev, (void*)d_ainv64, (void*)d_ainv32, (void*)d_rhs, (void*)d_dst, (void*)d_genB,
                    (void*)d_genBr})
        if (p) {
            if (pool)
                pool->release(p);
            else
                (void)hipFree(p);
        }
    pinned_put(h_pinned);
}

template <typename T>
static T* upload(const T* src, size_t count, DevicePool* pool = nullptr) {
    T* d = nullptr;
    if (pool) {
        d = static_cast<T*>(pool->alloc(std::max<size_t>(count, 1) * sizeof(T)));
    } else {
        hipError_t e = hipMalloc(&d, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(SG_ERR_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
        }
    }
    if (count && src) SG_HIP(hipMemcpy(d, src, count * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

// Host-side data of member b (coefficient modes, scalars, multigrid
// constants, coarse inverse) into the handle's host arrays, and the nonzero
// right-hand-side columns of the member into rb ([2][nt][nodes]).
static void fill_member(Handle* h, int b, const sg_problem& p, double* rb) {
    const Shape& s = h->s;
    const sg_options& opt = h->opt;
    const int M = s.M, n = s.n;
    const size_t cm = (size_t)(M + 1) * n * n;
    std::vector<double> c = coefficient_modes(p);
    std::copy(c.begin(), c.end(), h->coef_host.begin() + cm * b);
    MemberDev& md = h->mem_host[b];
    md.beta = p.beta;
    md.gamma = p.gamma;
    md.hg = 1.0 + p.gamma;
    md.c0 = c[0];
    const double sq = std::sqrt((1.0 + p.gamma) / p.beta);
    if (!s.time) {
        md.tau = 1.0;
        md.a1 = md.c0;          // A-tilde_1 = A_1 + sqrt((1+gamma)/beta) M  (eq. mathcalZ)
        md.b1 = sq;
        md.off_scale = 1.0;
    } else {
        md.tau = p.T / s.nt;    // A-hat_1 = (1 + tau sqrt((1+gamma)/beta)) M + tau A_1  (eq. A_hat)
        md.a1 = md.tau * md.c0;
        md.b1 = 1.0 + md.tau * sq;
        md.off_scale = md.tau;
    }
    for (int l = 0; l < s.nlev_mg; ++l) {
        LevelDev& L = h->lev_host[(size_t)b * kMaxLevels + l];
        const int m = s.mg_n[l];
        const double hh = 1.0 / m;
        L.wc = md.a1 * 8.0 / 3.0 + md.b1 * 16.0 * hh * hh / 36.0;
        L.we = -md.a1 / 3.0 + md.b1 * 4.0 * hh * hh / 36.0;
        L.wd = -md.a1 / 3.0 + md.b1 * hh * hh / 36.0;
        L.dinv = 1.0 / L.wc;
        const double lmax = lambda_max(m, md.a1, md.b1);
        smoother_coeffs(lmax, opt.gmg_pre, L.pre);
        smoother_coeffs(lmax, opt.gmg_post, L.post);
    }
    coarse_inverse(md.a1, md.b1, h->ainv_host.data() + (size_t)b * kCoarsePad * kCoarsePad);

    // right-hand side: b_y = tau D_t (M_full y_d)_interior in chaos column 0;
    // time with y0: b_lambda(t=0, j=0) = -(M_II y0)
    const double hh = 1.0 / n;
    const double w = hh * hh / 36.0;
    const int N1 = n + 1;
    for (int t = 0; t < s.nt; ++t) {
        const double* yd = p.y_target + (size_t)t * s.nodes;
        const double Dt = (s.time && (t == 0 || t == s.nt - 1)) ? 0.5 : 1.0;
        const double f = md.tau * Dt;
        for (int iy = 1; iy < n; ++iy)
            for (int ix = 1; ix < n; ++ix) {
                const int q = iy * N1 + ix;
                const double v = 16.0 * yd[q] + 4.0 * (yd[q - 1] + yd[q + 1] + yd[q - N1] + yd[q + N1]) +
                                 (yd[q - N1 - 1] + yd[q - N1 + 1] + yd[q + N1 - 1] + yd[q + N1 + 1]);
                rb[(size_t)t * s.nodes + q] = f * w * v;
            }
    }
    if (s.time && p.y0) {
        double* rl = rb + (size_t)s.nt * s.nodes;   // adjoint block, t = 0
        for (int iy = 1; iy < n; ++iy)
            for (int ix = 1; ix < n; ++ix) {
                auto y0i = [&](int jx, int jy) {
                    return (jx < 1 || jx > n - 1 || jy < 1 || jy > n - 1) ? 0.0 : p.y0[jy * N1 + jx];
                };
                const double v = 16.0 * y0i(ix, iy) +
                                 4.0 * (y0i(ix - 1, iy) + y0i(ix + 1, iy) + y0i(ix, iy - 1) + y0i(ix, iy + 1)) +
                                 (y0i(ix - 1, iy - 1) + y0i(ix + 1, iy - 1) + y0i(ix - 1, iy + 1) +
                                  y0i(ix + 1, iy + 1));
                rl[iy * N1 + ix] = -w * v;
            }
    }
}

// Element couplings of member b (log-normal field), computed on the host and
// copied to the member's slices of the device tables (synchronously).
static void upload_lognormal_member(Handle& h, int b, const sg_problem& p) {
    const Shape& s = h.s;
    std::vector<double> H, kappa;
    int nA = 0;
    lognormal_tables(p, s.nxi, h.ht.alpha, H, kappa, nA);
    const size_t per = (size_t)s.n * s.n * s.nxi * s.nxi;
    std::vector<double> B(per);
    lognormal_element_matrices(s.n, s.nxi, nA, nA, H, kappa, B.data());
    SG_HIP(hipMemcpy(h.d_genB + per * b, B.data(), sizeof(double) * per, hipMemcpyHostToDevice));
    if (h.d_genBr) {
        lognormal_element_matrices(s.n, s.nxi, nA, h.trunc_r(), H, kappa, B.data());
        SG_HIP(hipMemcpy(h.d_genBr + per * b, B.data(), sizeof(double) * per, hipMemcpyHostToDevice));
    }
}

void set_member(Handle& h, int b, const sg_problem& p) {
    const Shape& s = h.s;
    if (b < 0 || b >= h.B) throw Error(SG_ERR_INVALID, "member index out of range");
    validate(&p, 1, &h.opt);
    if (p.n != s.n || p.M != s.M || p.P != s.P || (p.n_t >= 2 ? p.n_t : 1) != s.nt || p.field != s.field)
        throw Error(SG_ERR_INVALID, "a member's problem must have the handle's n, M, P, n_t and field model");
    if (s.field == SG_FIELD_LOGNORMAL) {
        SG_HIP(hipStreamSynchronize(h.stream));     // the tables may be in use by earlier launches
        upload_lognormal_member(h, b, p);
    }
    const size_t rcols = (size_t)2 * s.nt * s.nodes;
    std::vector<double> rb(rcols, 0.0);
    fill_member(&h, b, p, rb.data());
    hipStream_t st = h.stream;
    const size_t cm = (size_t)(s.M + 1) * s.n * s.n;
    std::vector<float> c32(h.coef_host.begin() + cm * b, h.coef_host.begin() + cm * (b + 1));
    const size_t ca = (size_t)kCoarsePad * kCoarsePad;
    std::vector<float> a32(h.ainv_host.begin() + ca * b, h.ainv_host.begin() + ca * (b + 1));
    SG_HIP(hipMemcpyAsync(h.d_coef64 + cm * b, h.coef_host.data() + cm * b, sizeof(double) * cm,
                          hipMemcpyHostToDevice, st));
    SG_HIP(hipMemcpyAsync(h.d_coef32 + cm * b, c32.data(), sizeof(float) * cm, hipMemcpyHostToDevice, st));
    SG_HIP(hipMemcpyAsync(h.d_mem + b, h.mem_host.data() + b, sizeof(MemberDev), hipMemcpyHostToDevice, st));
    SG_HIP(hipMemcpyAsync(h.d_lev + (size_t)b * kMaxLevels, h.lev_host.data() + (size_t)b * kMaxLevels,
                          sizeof(LevelDev) * kMaxLevels, hipMemcpyHostToDevice, st));
    SG_HIP(hipMemcpyAsync(h.d_ainv64 + ca * b, h.ainv_host.data() + ca * b, sizeof(double) * ca,
                          hipMemcpyHostToDevice, st));
    SG_HIP(hipMemcpyAsync(h.d_ainv32 + ca * b, a32.data(), sizeof(float) * ca, hipMemcpyHostToDevice, st));
    const int64_t kkt = 3 * s.blk;
    launch_fill_zero<double>(h.d_rhs + (size_t)b * kkt, kkt, st);
    for (int v = 0; v < 2; ++v)
        SG_HIP(hipMemcpy2DAsync(h.d_rhs + (size_t)b * kkt + (size_t)(2 * v) * s.blk, sizeof(double) * s.tstride,
                                rb.data() + (size_t)v * s.nt * s.nodes, sizeof(double) * s.nodes,
                                sizeof(double) * s.nodes, s.nt, hipMemcpyHostToDevice, st));
    SG_HIP(hipStreamSynchronize(st));   // the host arrays above go out of scope
}

std::unique_ptr<Handle> build_handle(const sg_problem* probs, int count, const sg_options* opt_in, hipStream_t st,
                                     DevicePool* pool) {
    auto t0 = std::chrono::steady_clock::now();
    sg_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        default_options(&opt);
    validate(probs, count, &opt);

    auto h = std::make_unique<Handle>();
    h->opt = opt;
    h->B = count;
    h->stream = st;
    h->pool = pool;
    h->ws.set_pool(pool);
    SG_HIP(hipGetDevice(&h->device));
    {
        // the fused multigrid tail keeps every level up to 64 intervals per side and
        // the coarse inverse in LDS (141 KiB in FP64); with less LDS per workgroup
        // it starts at 32
        int lds = 0;
        SG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
        h->mg_tail_max = lds >= 144 * 1024 ? 64 : 32;
    }
    const sg_problem& p0 = probs[0];
    Shape& s = h->s;
    s.n = p0.n;
    s.M = p0.M;
    s.P = p0.P;
    s.time = p0.n_t >= 2;
    s.nt = s.time ? p0.n_t : 1;
    s.nxi = binom(s.M + s.P, s.P);
    s.nodes = (int64_t)(s.n + 1) * (s.n + 1);
    s.tstride = (int64_t)s.nxi * s.nodes;
    s.blk = (int64_t)s.nt * s.tstride;
    for (int d = 0; d <= s.P + 1; ++d) s.off[d] = d == 0 ? 0 : binom(s.M + d - 1, d - 1);
    s.nlev_mg = 0;
    for (int m = s.n; m >= kCoarseN; m /= 2) s.mg_n[s.nlev_mg++] = m;
    s.field = p0.field;
    s.nA = s.field == SG_FIELD_LOGNORMAL ? binom(s.M + 2 * s.P, 2 * s.P) : s.M + 1;

    // multi-index set and triple-product neighbour table:
    // E[psi_{e_k} psi_a psi_{a+e_k}] = sqrt(3) m / sqrt(4 m^2 - 1), m = a_k + 1
    // (three-term recurrence of orthonormal Legendre polynomials).
    const int M = s.M, nxi = s.nxi;
    h->ht.alpha = multi_indices(M, s.P);
    std::map<std::vector<int32_t>, int> index;
    for (int j = 0; j < nxi; ++j)
        index[std::vector<int32_t>(h->ht.alpha.begin() + (size_t)j * M, h->ht.alpha.begin() + (size_t)(j + 1) * M)] = j;
    h->ht.nbr_idx.assign((size_t)nxi * M * 2, -1);
    h->ht.nbr_val.assign((size_t)nxi * M * 2, 0.0);
    for (int j = 0; j < nxi; ++j) {
        std::vector<int32_t> a(h->ht.alpha.begin() + (size_t)j * M, h->ht.alpha.begin() + (size_t)(j + 1) * M);
        for (int k = 0; k < M; ++k) {
            const size_t slot = ((size_t)j * M + k) * 2;
            if (a[k] > 0) {
                std::vector<int32_t> b = a;
                b[k] -= 1;
                const double m = a[k];
                h->ht.nbr_idx[slot] = index.at(b);
                h->ht.nbr_val[slot] = std::sqrt(3.0) * m / std::sqrt(4.0 * m * m - 1.0);
            }
            std::vector<int32_t> b = a;
            b[k] += 1;
            auto it = index.find(b);
            if (it != index.end()) {
                const double m = a[k] + 1;
                h->ht.nbr_idx[slot + 1] = it->second;
                h->ht.nbr_val[slot + 1] = std::sqrt(3.0) * m / std::sqrt(4.0 * m * m - 1.0);
            }
        }
    }

    // members: coefficients, scalars, multigrid constants, right-hand sides
    const int n = s.n;
    const size_t cm = (size_t)(M + 1) * n * n;
    h->coef_host.resize(cm * count);
    h->mem_host.resize(count);
    h->lev_host.assign((size_t)count * kMaxLevels, LevelDev{});
    h->ainv_host.resize((size_t)count * kCoarsePad * kCoarsePad);
    const int64_t kkt = 3 * s.blk;
    const size_t rcols = (size_t)2 * s.nt * s.nodes;    // per member: state and adjoint column 0, every t
    h->rhs_host.assign((size_t)count * rcols, 0.0);
    for (int b = 0; b < count; ++b) fill_member(h.get(), b, probs[b], h->rhs_host.data() + (size_t)b * rcols);

    // upload
    h->d_nbr_idx = upload(h->ht.nbr_idx.data(), h->ht.nbr_idx.size(), pool);
    h->d_nbr_val = upload(h->ht.nbr_val.data(), h->ht.nbr_val.size(), pool);
    h->d_coef64 = upload(h->coef_host.data(), h->coef_host.size(), pool);
    {
        std::vector<float> c32(h->coef_host.begin(), h->coef_host.end());
        h->d_coef32 = upload(c32.data(), c32.size(), pool);
    }
    h->d_mem = upload(h->mem_host.data(), h->mem_host.size(), pool);
    h->d_lev = upload(h->lev_host.data(), h->lev_host.size(), pool);
    h->d_ainv64 = upload(h->ainv_host.data(), h->ainv_host.size(), pool);
    {
        std::vector<float> a32(h->ainv_host.begin(), h->ainv_host.end());
        h->d_ainv32 = upload(a32.data(), a32.size(), pool);
    }
    {
        // sine-transform tables of the exact solves: sin(pi m / n), m < 2n, then
        // the 1D stiffness and mass eigenvalues k_p = 4n sin^2(pi p / 2n),
        // m_p = (2 + cos(pi p / n)) / (3n), p = 0..n
        std::vector<double> t((size_t)2 * n + 2 * (n + 1));
        for (int m = 0; m < 2 * n; ++m) t[m] = std::sin(M_PI * (double)m / n);
        for (int q = 0; q <= n; ++q) {
            const double sh = std::sin(M_PI * q / (2.0 * n));
            t[2 * n + q] = 4.0 * n * sh * sh;
            t[2 * n + (n + 1) + q] = (2.0 + std::cos(M_PI * q / n)) / (3.0 * n);
        }
        h->d_dst = upload(t.data(), t.size(), pool);
    }
    if (s.field == SG_FIELD_LOGNORMAL) {
        const size_t per = (size_t)n * n * s.nxi * s.nxi;
        const int r = h->trunc_r();
        h->d_genB = upload<double>(nullptr, per * count, pool);
        if (r < s.nA) h->d_genBr = upload<double>(nullptr, per * count, pool);
        for (int b = 0; b < count; ++b) upload_lognormal_member(*h, b, probs[b]);
    }
    {
        // right-hand sides: zero everywhere but chaos column 0 of the state
        // and adjoint blocks, so only those columns cross the bus
        double* cols = upload(h->rhs_host.data(), h->rhs_host.size(), pool);
        h->d_rhs = upload<double>(nullptr, (size_t)count * kkt, pool);
        launch_fill_zero<double>(h->d_rhs, (int64_t)count * kkt, st);
        for (int b = 0; b < count; ++b)
            for (int v = 0; v < 2; ++v)
                SG_HIP(hipMemcpy2DAsync(h->d_rhs + (size_t)b * kkt + (size_t)(2 * v) * s.blk,
                                        sizeof(double) * s.tstride, cols + ((size_t)b * 2 + v) * s.nt * s.nodes,
                                        sizeof(double) * s.nodes, sizeof(double) * s.nodes, s.nt,
                                        hipMemcpyDeviceToDevice, st));
        SG_HIP(hipStreamSynchronize(st));
        if (pool) pool->release(cols); else (void)hipFree(cols);
        h->rhs_host.clear();
        h->rhs_host.shrink_to_fit();
    }
    h->h_pinned = pinned_get();
    h->h_pinned_count = kPinnedDoubles;
    autotune(*h);
    SG_HIP(hipStreamSynchronize(h->stream));
    h->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return h;
}

}  // namespace sg
