// Solver orchestration on one HIP stream: operator and KKT applies, the
// block-diagonal preconditioner (Chebyshev mass solves, hierarchical
// Gauss-Seidel with multigrid inner solves), flexible GMRES with FP64 Arnoldi,
// and FP64 iterative refinement around an FP32 inner solve.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>

#include "handle.hpp"

namespace sg {

bool prof_begin(Handle& h, int kind, hipStream_t st) {
    if (h.prof.kind != kind || kind == SG_PROF_NONE) return false;
    if (h.prof.used == h.prof.ev.size()) {
        hipEvent_t a, b;
        SG_HIP(hipEventCreate(&a));
        SG_HIP(hipEventCreate(&b));
        h.prof.ev.push_back({a, b});
    }
    SG_HIP(hipEventRecord(h.prof.ev[h.prof.used].first, st));
    return true;
}

void prof_end(Handle& h, hipStream_t st, double bytes) {
    SG_HIP(hipEventRecord(h.prof.ev[h.prof.used].second, st));
    ++h.prof.used;
    h.prof.bytes += bytes;
}

double prof_collect_ms(Handle& h) {
    double total = 0.0;
    for (size_t i = 0; i < h.prof.used; ++i) {
        SG_HIP(hipEventSynchronize(h.prof.ev[i].second));
        float ms = 0.f;
        SG_HIP(hipEventElapsedTime(&ms, h.prof.ev[i].first, h.prof.ev[i].second));
        total += ms;
    }
    return total;
}

namespace {

template <typename T>
const char* tname() {
    return sizeof(T) == 8 ? "64" : "32";
}

// Column map for the degree-d columns of a field block stored with member stride `mstride`.
ColMap level_map(const Shape& s, int d, int64_t mstride) {
    ColMap m;
    m.mstride = mstride;
    m.tstride = s.tstride;
    m.nodes = s.nodes;
    m.L = s.off[d + 1] - s.off[d];
    m.nt = s.nt;
    m.j0 = s.off[d];
    return m;
}

ColMap block_map(const Shape& s, int64_t mstride) {
    ColMap m;
    m.mstride = mstride;
    m.tstride = s.tstride;
    m.nodes = s.nodes;
    m.L = s.nxi;
    m.nt = s.nt;
    m.j0 = 0;
    return m;
}

// One multigrid V-cycle for the columns of degree level d (all members, all
// time steps): b (level-d columns through bmap) -> x (through xmap).  Column c
// uses the constants of member c / cpm (cpm = ncols when all columns share
// member 0).
// Levels with at most mg_tail_max intervals per side (and the direct solve)
// run in one fused launch; the finer levels have a down and an up launch each.
// Returns the first level handled by the fused tail (or the direct solve) and
// whether the tail is used.
int mg_first_fused(const Handle& h, bool& tail) {
    const Shape& s = h.s;
    const int nl = s.nlev_mg;
    int l0 = 0;
    while (l0 < nl - 1 && s.mg_n[l0] > h.mg_tail_max) ++l0;
    tail = l0 < nl - 1;
    return tail ? l0 : nl - 1;
}

// Per-level multigrid scratch of a V-cycle over ncols columns: bs (restricted
// right-hand side, l >= 1), xf (after post-smoothing, l >= 1; level 0 writes
// to x), xp (pre-smoothed iterate, levels run by the down/up kernels); xs only
// for the coarsest level solved directly.
template <typename T>
void mg_buffers(Handle& h, int ncols, std::vector<T*>& xs, std::vector<T*>& bs, std::vector<T*>& xf,
                std::vector<T*>& xp, std::vector<ColMap>& cm) {
    const Shape& s = h.s;
    const int nl = s.nlev_mg;
    bool tail = false;
    const int lc = mg_first_fused(h, tail);
    xs.assign(nl, nullptr);
    bs.assign(nl, nullptr);
    xf.assign(nl, nullptr);
    xp.assign(nl, nullptr);
    cm.assign(nl, ColMap{});
    for (int l = 0; l <= lc; ++l) {
        const int m = s.mg_n[l];
        const int64_t nodes = (int64_t)(m + 1) * (m + 1);
        const size_t cnt = (size_t)ncols * nodes;
        const std::string tag = std::string("mg") + tname<T>() + "_" + std::to_string(l);
        cm[l] = contiguous_cols(ncols, nodes);
        if (l == lc && !tail) xs[l] = h.ws.get_t<T>(tag + "_xs", cnt);
        if (l < lc) xp[l] = h.ws.get_t<T>(tag + "_xp", cnt);
        if (l > 0) {
            bs[l] = h.ws.get_t<T>(tag + "_bs", cnt);
            xf[l] = h.ws.get_t<T>(tag + "_xf", cnt);
        }
    }
}

// One multigrid V-cycle for the columns of degree level d (all members, all
// time steps): b (level-d columns through bmap) -> x (through xmap).  Column c
// uses the constants of member c / cpm (cpm = ncols when all columns share
// member 0).
template <typename T>
void vcycle(Handle& h, const T* b, ColMap bmap, T* x, ColMap xmap, int ncols, int cpm, int cpv, hipStream_t st) {
    const Shape& s = h.s;
    const LevelDev* lev = h.d_lev;
    const int nl = s.nlev_mg;
    const int npre = h.opt.gmg_pre, npost = h.opt.gmg_post;
    if (nl == 1) {
        launch_mg_coarse<T>(h.ainv<T>(), b, bmap, x, xmap, ncols, cpm, st);
        return;
    }
    bool tail = false;
    const int lc = mg_first_fused(h, tail);
    std::vector<T*> xs, bs, xf, xp;
    std::vector<ColMap> cm;
    mg_buffers<T>(h, ncols, xs, bs, xf, xp, cm);
    for (int l = 0; l < lc; ++l) {
        const int m = s.mg_n[l];
        const double nodes = (double)(m + 1) * (m + 1);
        const bool tp = l == 0 && prof_begin(h, SG_PROF_MG_SMOOTH, st);
        launch_mg_down<T>(m, lev, l, npre, l == 0 ? b : bs[l], l == 0 ? bmap : cm[l], bs[l + 1], xp[l], ncols, cpm,
                          h.active, cpv, st);
        if (tp) prof_end(h, st, sizeof(T) * ncols * nodes * 2.25);   // read b, write the iterate and b_coarse
    }
    const T* e;
    if (tail) {
        T* out = lc == 0 ? x : xf[lc];
        const bool tp = prof_begin(h, SG_PROF_MG_TAIL, st);
        launch_mg_tail<T>(s.mg_n[lc], lev, lc, npre, npost, lc == 0 ? b : bs[lc], lc == 0 ? bmap : cm[lc], out,
                          lc == 0 ? xmap : cm[lc], h.ainv<T>(), ncols, cpm, h.active, cpv, st);
        // algorithmic bytes: read b, write x at the first fused level
        if (tp) prof_end(h, st, 2.0 * sizeof(T) * ncols * (double)(s.mg_n[lc] + 1) * (s.mg_n[lc] + 1));
        e = out;
    } else {
        launch_mg_coarse<T>(h.ainv<T>(), bs[nl - 1], cm[nl - 1], xs[nl - 1], cm[nl - 1], ncols, cpm, st);
        e = xs[nl - 1];
    }
    for (int l = lc - 1; l >= 0; --l) {
        const int m = s.mg_n[l];
        const double nodes = (double)(m + 1) * (m + 1);
        T* out = l == 0 ? x : xf[l];
        const bool tp = l == 0 && prof_begin(h, SG_PROF_MG_UP, st);
        launch_mg_up<T>(m, lev, l, npost, e, l == 0 ? b : bs[l], l == 0 ? bmap : cm[l], xp[l], out,
                        l == 0 ? xmap : cm[l], ncols, cpm, h.active, cpv, st);
        if (tp) prof_end(h, st, sizeof(T) * ncols * nodes * 3.25);  // read b, the iterate, e_coarse; write x
        e = out;
    }
}

// FP64 scratch of the sine-transform solves: two buffers of the largest
// column count a preconditioner application of nvec vectors uses (the mass
// blocks, 2 n_t n_xi columns per vector, or the widest degree level).
void dst_scratch(Handle& h, int nvec, double*& s1, double*& s2) {
    const Shape& s = h.s;
    int lmax = 0;
    for (int d = 0; d <= s.P; ++d) lmax = std::max(lmax, s.off[d + 1] - s.off[d]);
    const size_t cols = (size_t)nvec * s.nt * std::max(2 * s.nxi, lmax);
    s1 = h.ws.get_t<double>("dst1", cols * s.nodes);
    s2 = h.ws.get_t<double>("dst2", cols * s.nodes);
}

// Solves with the mean block A-tilde_1 (eq. mathcalZ) / A-hat_1 (eq. A_hat)
// on ncols columns: one multigrid V-cycle, or exactly by the sine transform.
template <typename T>
void mean_solve(Handle& h, const T* b, ColMap bmap, T* x, ColMap xmap, int ncols, int cpm, int cpv, int nvec,
                hipStream_t st) {
    if (h.opt.mean_solver == SG_MEAN_EXACT) {
        double *s1, *s2;
        dst_scratch(h, nvec, s1, s2);
        const Shape& s = h.s;
        launch_dst_solve<T>(s.n, 1, h.d_mem, 0, h.d_dst, h.d_dst + 2 * s.n, b, bmap, x, xmap, ncols, cpm, s.nt,
                            s.nxi, (int)s.time, s1, s2, h.active, cpv, st);
        return;
    }
    vcycle<T>(h, b, bmap, x, xmap, ncols, cpm, cpv, st);
}

// hGS (Algorithm 1): V = Z_r^{-1}-approximation applied to R, zero initial
// guess, forward sweep over degrees 0..P then backward P-1..0.  R and V are
// field blocks with member strides rms / vms; nmem members.
template <typename T>
void hgs(Handle& h, const T* R, int64_t rms, T* V, int64_t vms, int nmem, bool shared, hipStream_t st) {
    const Shape& s = h.s;
    const OpDev op = h.op<T>(shared);
    const uint32_t mask = h.modes_mask();
    T* Bs = h.ws.get_t<T>(std::string("hgsB") + tname<T>(), (size_t)nmem * s.blk);
    const ColMap vfull = block_map(s, vms);
    for (int d = 0; d <= s.P; ++d) {
        const ColMap rm = level_map(s, d, rms), bm = level_map(s, d, s.blk), vm = level_map(s, d, vms);
        const int L = s.off[d + 1] - s.off[d];
        const int Ln = d > 0 ? s.off[d] - s.off[d - 1] : 0;
        if (d == 0) {
            // degree 0 has no lower level: its right-hand side is R_(0) itself (the
            // multigrid reads interior nodes only), solved from R directly
            mean_solve<T>(h, R, rm, V, vm, L * s.nt * nmem, shared ? L * s.nt * nmem : L * s.nt, L * s.nt, nmem, st);
            continue;
        }
        const bool tp = prof_begin(h, SG_PROF_HGS_RHS, st);
        launch_hgs_rhs<T>(s, op, d, mask, 1, 0, R, rm, V, vfull, Bs, bm, nmem, st);
        if (tp) prof_end(h, st, (double)sizeof(T) * (2 * L + (mask ? Ln : 0)) * s.nodes * s.nt * nmem);
        mean_solve<T>(h, Bs, bm, V, vm, L * s.nt * nmem, shared ? L * s.nt * nmem : L * s.nt, L * s.nt, nmem, st);
    }
    if (mask == 0) return;   // mean-based: the backward sweep repeats the forward solves exactly
    for (int d = s.P - 1; d >= 0; --d) {
        const ColMap bm = level_map(s, d, s.blk), vm = level_map(s, d, vms);
        const int L = s.off[d + 1] - s.off[d];
        const int Lu = s.off[d + 2] - s.off[d + 1];
        const bool tp = prof_begin(h, SG_PROF_HGS_RHS, st);
        // base: the forward sweep's right-hand side of level d (R_(0) itself at d = 0)
        if (d == 0)
            launch_hgs_rhs<T>(s, op, d, mask, 0, 1, R, level_map(s, 0, rms), V, vfull, Bs, bm, nmem, st);
        else
            launch_hgs_rhs<T>(s, op, d, mask, 0, 1, Bs, bm, V, vfull, Bs, bm, nmem, st);
        if (tp) prof_end(h, st, (double)sizeof(T) * (2 * L + Lu) * s.nodes * s.nt * nmem);
        mean_solve<T>(h, Bs, bm, V, vm, L * s.nt * nmem, shared ? L * s.nt * nmem : L * s.nt, L * s.nt, nmem, st);
    }
}

}  // namespace

template <typename T>
void operator_apply(Handle& h, const T* x, T* y, int nvec, bool shared, hipStream_t st) {
    launch_sg_apply<T>(h.s, h.op<T>(shared), x, y, nvec, 0xffffffffu, st);
}

template <typename T>
void kkt_apply(Handle& h, const T* x, T* y, int nvec, bool shared, hipStream_t st) {
    const bool tp = prof_begin(h, SG_PROF_KKT_APPLY, st);
    if (h.s.field == SG_FIELD_LOGNORMAL) {
        T* T1 = h.ws.get_t<T>(std::string("genT1") + tname<T>(), (size_t)nvec * h.s.blk);
        T* T2 = h.ws.get_t<T>(std::string("genT2") + tname<T>(), (size_t)nvec * h.s.blk);
        launch_gen_kkt<T>(h.s, h.op<T>(shared), x, y, T1, T2, nvec, st);
    } else {
        launch_kkt_apply<T>(h.s, h.op<T>(shared), x, y, nvec, st);
    }
    // algorithmic bytes: read the three fields, write the three results, read the coefficient modes
    if (tp)
        prof_end(h, st,
                 (double)sizeof(T) * nvec * (6.0 * h.s.blk + (shared ? 1.0 / nvec : 1.0) * (h.s.M + 1) * h.s.n * h.s.n));
}

// Z^{-1} of the Schur block on nvec field blocks: Algorithm 5 with N =
// richardson_steps from a zero initial guess, each step preconditioned by
// one hGS (Algorithm 1): X <- X + hGS(R - Z_r X), Z_r = I (x) A-tilde_1 +
// off_scale sum_{k<r} G_k (x) K_k.  N = 1 is one hGS, written to V directly.
template <typename T>
void zinv(Handle& h, const T* R, int64_t rms, T* V, int64_t vms, int nvec, bool shared, hipStream_t st) {
    const int N = h.opt.richardson_steps;
    if (N <= 1) {
        hgs<T>(h, R, rms, V, vms, nvec, shared, st);
        return;
    }
    const Shape& s = h.s;
    const size_t cnt = (size_t)nvec * s.blk;
    T* X = h.ws.get_t<T>(std::string("richX") + tname<T>(), cnt);
    T* Y = h.ws.get_t<T>(std::string("richY") + tname<T>(), cnt);
    T* Rr = h.ws.get_t<T>(std::string("richR") + tname<T>(), cnt);
    T* D = h.ws.get_t<T>(std::string("richD") + tname<T>(), cnt);
    const ColMap bm = block_map(s, s.blk), rm = block_map(s, rms), vm = block_map(s, vms);
    const int ncols = nvec * s.nt * s.nxi, cpv = s.nt * s.nxi;
    const OpDev op = h.op<T>(shared);
    hgs<T>(h, R, rms, X, s.blk, nvec, shared, st);
    for (int k = 1; k < N; ++k) {
        launch_sg_apply<T>(s, op, X, Y, nvec, h.modes_mask(), st);
        launch_z_residual<T>(s.n, R, rm, Y, X, bm, Rr, bm, h.d_mem, ncols, cpv, shared ? 1 : 0, h.active, st);
        hgs<T>(h, Rr, s.blk, D, s.blk, nvec, shared, st);
        if (k + 1 < N)
            launch_cols_add<T>(s.nodes, X, bm, D, bm, X, bm, ncols, cpv, h.active, st);
        else
            launch_cols_add<T>(s.nodes, X, bm, D, bm, V, vm, ncols, cpv, h.active, st);
    }
}

// hGSoc (Algorithms 2-3; on the all-at-once time-dependent system applied to
// every time step at once, Algorithm 4): one forward (degrees 0..P) and one
// backward (P-1..0) sweep over the degree levels of the whole KKT vector, zero
// initial guess.  At level d the state and adjoint rows take the KKT couplings to the
// other levels with their current values (R^Y_d + sum_k K_k Lambda and R^L_d +
// sum_k K_k Y over the kept modes; the control row has none), and the level
// is solved with the block-diagonal preconditioner restricted to its chaos
// columns: h^gamma_j M and beta M by Chebyshev, the adjoint by A-tilde_1^{-1}
// h^gamma_j M A-tilde_1^{-1} (the Schur-type reading of P-tilde; the printed
// third block A-tilde_1 stagnates).  As in Alg. 1 the backward sweep reuses
// the forward right-hand side of each level and adds the upper levels.  For a
// time step t the level blocks are tau D_tt h^gamma_j M, beta tau D_tt M and
// A-hat_1 (tau D_tt h^gamma_j M)^{-1} A-hat_1 and the couplings carry tau
// (the member's off_scale); the couplings to the neighbouring steps are left
// out, so the steps are independent.
template <typename T>
void hgsoc_apply(Handle& h, const T* r, T* z, int nvec, bool shared, hipStream_t st) {
    const Shape& s = h.s;
    OpDev op = h.op<T>(shared);
    op.off_sign = -1.0;                      // the couplings enter the level right-hand sides with +
    const uint32_t mask = h.modes_mask();
    const int64_t kkt = 3 * s.blk;
    const size_t cnt = (size_t)nvec * s.blk;
    T* BY = h.ws.get_t<T>(std::string("socY") + tname<T>(), cnt);
    T* BL = h.ws.get_t<T>(std::string("socL") + tname<T>(), cnt);
    T* T1 = h.ws.get_t<T>(std::string("socT1") + tname<T>(), cnt);
    T* T2 = h.ws.get_t<T>(std::string("socT2") + tname<T>(), cnt);
    const ColMap vfull = block_map(s, kkt);
    auto level = [&](int d, bool fwd) {
        const ColMap rm = level_map(s, d, kkt), bm = level_map(s, d, s.blk);
        const int L = s.off[d + 1] - s.off[d];
        const int ncols = L * s.nt * nvec, cpm = shared ? ncols : L * s.nt, cpv = L * s.nt;
        // right-hand sides of the state and adjoint rows (base: the residual, or
        // backward the forward right-hand side of this level)
        const T* bY = r;
        const T* bL = r + 2 * s.blk;
        ColMap bYm = rm, bLm = rm;
        if (mask != 0 && (d > 0 || !fwd)) {
            const bool from_r = fwd || d == 0;
            launch_hgs_rhs<T>(s, op, d, mask, fwd ? 1 : 0, fwd ? 0 : 1, from_r ? r : BY, from_r ? rm : bm,
                              z + 2 * s.blk, vfull, BY, bm, nvec, st);
            launch_hgs_rhs<T>(s, op, d, mask, fwd ? 1 : 0, fwd ? 0 : 1, from_r ? r + 2 * s.blk : BL, from_r ? rm : bm,
                              z, vfull, BL, bm, nvec, st);
            bY = BY;
            bL = BL;
            bYm = bLm = bm;
        }
        // state and control columns of the level (L consecutive columns in each
        // time step, n_xi apart): Chebyshev with the block scalings
        const bool yb = bY == BY;
        if (!launch_mass_cheb_cols<T>(s, op, yb ? BY : r, yb ? s.blk : kkt, z, kkt, s.off[d], L, s.nt, s.nxi, nvec,
                                      h.opt.cheb_steps, st) ||
            !launch_mass_cheb_cols<T>(s, op, r, kkt, z, kkt, s.nt * s.nxi + s.off[d], L, s.nt, s.nxi, nvec,
                                      h.opt.cheb_steps, st))
            throw Error(SG_ERR_INVALID, "hGSoc needs cheb_steps in [1, 9]");
        // adjoint columns: A-tilde_1^{-1} h^gamma_j M A-tilde_1^{-1}
        mean_solve<T>(h, bL, bLm, T1, bm, ncols, cpm, cpv, nvec, st);
        launch_mass_scaled<T>(s, op, T1, bm, T2, bm, ncols, nvec, st);
        mean_solve<T>(h, T2, bm, z + 2 * s.blk, rm, ncols, cpm, cpv, nvec, st);
    };
    for (int d = 0; d <= s.P; ++d) level(d, true);
    if (mask == 0) return;   // mean-based: the backward sweep repeats the forward solves exactly
    for (int d = s.P - 1; d >= 0; --d) level(d, false);
}

// Block-diagonal preconditioner (eq. stoch-prec / eq. precon for time).
template <typename T>
void precond_apply(Handle& h, const T* r, T* z, int nvec, bool shared, hipStream_t st) {
    if (h.opt.precond == SG_PRECOND_HGSOC) {
        hgsoc_apply<T>(h, r, z, nvec, shared, st);
        return;
    }
    const Shape& s = h.s;
    const OpDev op = h.op<T>(shared);
    const int64_t kkt = 3 * s.blk;
    // state and control blocks: Chebyshev semi-iteration on M with block
    // scalings, or (cheb_steps = 0) exact solves by the sine transform
    const bool tp = prof_begin(h, SG_PROF_MASS_CHEB, st);
    if (h.opt.cheb_steps == 0) {
        double *s1, *s2;
        dst_scratch(h, nvec, s1, s2);
        ColMap ym;       // columns [y | u] of each vector: n_t n_xi state columns, then the control columns
        ym.mstride = kkt;
        ym.tstride = 0;
        ym.nodes = s.nodes;
        ym.L = 2 * s.nt * s.nxi;
        ym.nt = 1;
        ym.j0 = 0;
        launch_dst_solve<T>(s.n, 2, h.d_mem, shared ? 1 : 0, h.d_dst, h.d_dst + 2 * s.n, r, ym, z, ym,
                            nvec * 2 * s.nt * s.nxi, 1, s.nt, s.nxi, (int)s.time, s1, s2, h.active, ym.L, st);
    } else {
        // (the per-step Chebyshev kernel, used above 9 steps, needs two iterate buffers)
        const bool cheb_bufs = h.opt.cheb_steps > 9;
        T* A = cheb_bufs ? h.ws.get_t<T>(std::string("chebA") + tname<T>(), (size_t)nvec * 2 * s.blk) : nullptr;
        T* Bb = cheb_bufs ? h.ws.get_t<T>(std::string("chebB") + tname<T>(), (size_t)nvec * 2 * s.blk) : nullptr;
        launch_mass_cheb<T>(s, op, r, z, A, Bb, nvec, h.opt.cheb_steps, st);
    }
    if (tp) prof_end(h, st, 4.0 * sizeof(T) * nvec * (double)s.blk);   // read r_y, r_u; write z_y, z_u
    // adjoint block: S^{-1} r = Z^{-1} (tau D (x) M_gamma) Z^{-1} r
    T* V1 = h.ws.get_t<T>(std::string("schurV") + tname<T>(), (size_t)nvec * s.blk);
    T* W = h.ws.get_t<T>(std::string("schurW") + tname<T>(), (size_t)nvec * s.blk);
    zinv<T>(h, r + 2 * s.blk, kkt, V1, s.blk, nvec, shared, st);
    const ColMap vm = block_map(s, s.blk);
    launch_mass_scaled<T>(s, op, V1, vm, W, vm, nvec * s.nt * s.nxi, nvec, st);
    zinv<T>(h, W, s.blk, z + 2 * s.blk, kkt, nvec, shared, st);
}

// Every scratch buffer precond_apply<T> uses for nvec vectors, requested at
// its largest size (the multigrid levels are sized for the largest degree
// level), so that in arena mode a call that does not fit fails here, before
// any launch.
template <typename T>
void precond_reserve(Handle& h, int nvec) {
    const Shape& s = h.s;
    if (h.opt.cheb_steps > 9) {
        h.ws.get_t<T>(std::string("chebA") + tname<T>(), (size_t)nvec * 2 * s.blk);
        h.ws.get_t<T>(std::string("chebB") + tname<T>(), (size_t)nvec * 2 * s.blk);
    }
    h.ws.get_t<T>(std::string("schurV") + tname<T>(), (size_t)nvec * s.blk);
    h.ws.get_t<T>(std::string("schurW") + tname<T>(), (size_t)nvec * s.blk);
    h.ws.get_t<T>(std::string("hgsB") + tname<T>(), (size_t)nvec * s.blk);
    if (h.opt.cheb_steps == 0 || h.opt.mean_solver == SG_MEAN_EXACT) {
        double *s1, *s2;
        dst_scratch(h, nvec, s1, s2);
    }
    if (h.opt.richardson_steps > 1)
        for (const char* nm : {"richX", "richY", "richR", "richD"})
            h.ws.get_t<T>(std::string(nm) + tname<T>(), (size_t)nvec * s.blk);
    if (h.opt.precond == SG_PRECOND_HGSOC)
        for (const char* nm : {"socY", "socL", "socT1", "socT2"})
            h.ws.get_t<T>(std::string(nm) + tname<T>(), (size_t)nvec * s.blk);
    if (s.nlev_mg > 1) {
        int lmax = 0;
        for (int d = 0; d <= s.P; ++d) lmax = std::max(lmax, s.off[d + 1] - s.off[d]);
        std::vector<T*> xs, bs, xf, xp;
        std::vector<ColMap> cm;
        mg_buffers<T>(h, lmax * s.nt * nvec, xs, bs, xf, xp, cm);
    }
}

template void precond_reserve<double>(Handle&, int);
template void precond_reserve<float>(Handle&, int);
template void operator_apply<double>(Handle&, const double*, double*, int, bool, hipStream_t);
template void operator_apply<float>(Handle&, const float*, float*, int, bool, hipStream_t);
template void kkt_apply<double>(Handle&, const double*, double*, int, bool, hipStream_t);
template void kkt_apply<float>(Handle&, const float*, float*, int, bool, hipStream_t);
template void precond_apply<double>(Handle&, const double*, double*, int, bool, hipStream_t);
template void precond_apply<float>(Handle&, const float*, float*, int, bool, hipStream_t);

// ---------------------------------------------------------------------------
// Model of the algorithmic HBM bytes of a solve (sg_solve_info.bytes_moved):
// every launch counted as the streaming passes its kernels must make, each
// input and output node once, per member.
// ---------------------------------------------------------------------------
namespace {

// one mean-block solve of one column: a multigrid V-cycle reads b and writes
// the pre-smoothed iterate and the coarse right-hand side going down (2.25
// node passes), reads b, that iterate and the coarse correction and writes x
// going up (3.25), over levels shrinking by four (x 4/3); the sine-transform
// solve makes four FP64 passes, each reading and writing the column
double mean_solve_bytes(const Handle& h, double sz) {
    const double nodes = (double)h.s.nodes;
    if (h.opt.mean_solver == SG_MEAN_EXACT) return 8.0 * 8.0 * nodes;
    return sz * nodes * 5.5 * 4.0 / 3.0;
}

// one hGS sweep pair (Alg. 1) on one member's field block: the level
// right-hand sides and one mean-block solve per level column, forward and
// (unless mean-based) backward
double hgs_bytes(const Handle& h, double sz) {
    const Shape& s = h.s;
    const double col = sz * (double)s.nodes * s.nt;
    const bool back = h.modes_mask() != 0;
    double b = 0.0;
    for (int d = 0; d <= s.P; ++d) {
        const int L = s.off[d + 1] - s.off[d];
        const int Ln = d > 0 ? s.off[d] - s.off[d - 1] : 0;
        if (d > 0) b += (2.0 * L + (back ? Ln : 0)) * col;
        b += L * s.nt * mean_solve_bytes(h, sz);
    }
    if (!back) return b;
    for (int d = s.P - 1; d >= 0; --d) {
        const int L = s.off[d + 1] - s.off[d];
        const int Lu = s.off[d + 2] - s.off[d + 1];
        b += (2.0 * L + Lu) * col + L * s.nt * mean_solve_bytes(h, sz);
    }
    return b;
}

double model_operator_bytes(const Handle& h, double sz) {
    const Shape& s = h.s;
    double b = sz * (6.0 * s.blk + (s.M + 1.0) * s.n * s.n);
    if (s.field == SG_FIELD_LOGNORMAL) b += 2.0 * 8.0 * s.n * s.n * (double)s.nxi * s.nxi;   // element tables, two products
    return b;
}

double model_precond_bytes(const Handle& h, double sz) {
    const Shape& s = h.s;
    const double blk = (double)s.blk;
    // state and control blocks: read r, write z (Chebyshev, fused); the
    // sine-transform solves: four FP64 passes reading and writing each column
    double b = h.opt.cheb_steps == 0 ? 2.0 * 8.0 * 8.0 * blk : 4.0 * sz * blk;
    if (h.opt.precond == SG_PRECOND_HGSOC) {
        // coupled sweep: both right-hand sides, the state/control Chebyshev and two
        // mean-block solves with the scaled mass between them, per level column
        return b + 2.0 * hgs_bytes(h, sz) + 2.0 * sz * blk;
    }
    // Schur block: two Z^{-1} (each N hGS, and between them an SG apply, the
    // residual and the update), the scaled mass in the middle
    const int N = std::max(1, h.opt.richardson_steps);
    const double zinv = N * hgs_bytes(h, sz) + (N - 1) * (sz * 2.0 * blk + sz * 3.0 * blk + sz * 3.0 * blk);
    return b + 2.0 * zinv + 2.0 * sz * blk;
}

}  // namespace

// ---------------------------------------------------------------------------
// Flexible GMRES
// ---------------------------------------------------------------------------
namespace {

struct Krylov {
    Handle& h;
    int B;
    int m;                 // restart
    int64_t N;             // KKT vector length per member
    int nblk;
    hipStream_t st;
    void* V;               // [m+1][vs]: slot i holds the B member vectors back to back (double, or float if v32)
    int64_t vs;            // slot stride: B*N rounded up to 64 elements
    void* Z;               // [m][B][N] (double or float)
    bool z32;              // preconditioner in FP32, Z stored in FP32
    bool op32;             // KKT operator on Z_j from FP32 storage too (refinement inner cycles)
    bool v32;              // basis and w in FP32 storage as well (refinement inner cycles, DCGS2)
    double* zt;            // [B][N] FP64 copy of Z_j (z32 && !op32)
    double* w;             // [B][N]
    double* partial;       // [B][kSlots][nblk]
    KrylovDev kd;
    int* ctl;              // [4][B] device: active, iters, itmax, jend (one upload per cycle)
    float* v32buf;         // [B][N] FP32 staging (FP32 preconditioner on an FP64 basis)
    float* w32;            // [B][N] FP32 operator output (op32)

    // fp32_precond: Z in FP32; fp32_op: the operator on Z also from FP32
    // storage; fp32_basis (with fp32_op, DCGS2 only): V and w in FP32 too.
    Krylov(Handle& hh, bool fp32_precond, bool fp32_op, bool fp32_basis) : h(hh), st(hh.stream) {
        const Shape& s = h.s;
        B = h.B;
        m = h.opt.restart;
        N = 3 * s.blk;
        nblk = (int)std::min<int64_t>(4096, std::max<int64_t>(1, N / (256 * 16)));
        z32 = fp32_precond;
        op32 = fp32_precond && fp32_op;
        v32 = op32 && fp32_basis && h.opt.arnoldi == SG_ARNOLDI_DCGS2;
        vs = ((int64_t)B * N + 63) / 64 * 64;
        V = v32 ? (void*)h.ws.get_t<float>("kV32", (size_t)(m + 1) * vs) : (void*)h.ws.get_t<double>("kV", (size_t)(m + 1) * vs);
        Z = z32 ? (void*)h.ws.get_t<float>("kZ32", (size_t)m * B * N) : (void*)h.ws.get_t<double>("kZ", (size_t)m * B * N);
        w = v32 ? nullptr : h.ws.get_t<double>("kw", (size_t)B * N);
        partial = h.ws.get_t<double>("kpart", (size_t)B * kSlots * nblk);
        const int ld = m + 1;
        kd.H = h.ws.get_t<double>("kH", (size_t)B * ld * m);
        kd.cs = h.ws.get_t<double>("kcs", (size_t)B * m);
        kd.sn = h.ws.get_t<double>("ksn", (size_t)B * m);
        kd.g = h.ws.get_t<double>("kg", (size_t)B * ld);
        kd.h1 = h.ws.get_t<double>("kh1", (size_t)B * ld);
        kd.h2 = h.ws.get_t<double>("kh2", (size_t)B * ld);
        kd.nrm = h.ws.get_t<double>("knrm", (size_t)B);
        kd.y = h.ws.get_t<double>("ky", (size_t)B * m);
        kd.resid = h.ws.get_t<double>("kres", (size_t)B);
        ctl = h.ws.get_t<int>("kctl", (size_t)4 * B);
        kd.active = ctl;
        kd.iters = ctl + B;
        kd.itmax = ctl + 2 * B;
        kd.jend = ctl + 3 * B;
        kd.tol = h.ws.get_t<double>("ktol", (size_t)B);
        kd.dots = h.ws.get_t<double>("kdots", (size_t)B * kSlots);
        kd.scal = h.ws.get_t<double>("kscal", (size_t)B * 4);
        kd.pending = h.ws.get_t<int>("kpend", (size_t)B);
        kd.R = h.ws.get_t<double>("kR", (size_t)B * ld * ld);
        kd.coef = h.ws.get_t<double>("kcoef", (size_t)B * kSlots);
        v32buf = z32 && !v32 ? h.ws.get_t<float>("kv32", (size_t)B * N) : nullptr;
        w32 = op32 ? h.ws.get_t<float>("kw32", (size_t)B * N) : nullptr;
        zt = z32 && !op32 ? h.ws.get_t<double>("kzt", (size_t)B * N) : nullptr;
    }
    double* Vi(int i) { return (double*)V + (int64_t)i * vs; }
    float* Vi32(int i) { return (float*)V + (int64_t)i * vs; }

    // y = K x for all members (FP64, or through FP32 storage when fp32)
    void apply_op(const double* x, double* y, bool fp32) {
        if (!fp32) {
            kkt_apply<double>(h, x, y, B, B == 1, st);
        } else {
            float* xs = w32;   // staging: x in FP32, product in FP32
            float* ys = v32buf ? v32buf : h.ws.get_t<float>("kv32", (size_t)B * N);
            launch_cast_d2f(x, xs, (int64_t)B * N, st);
            kkt_apply<float>(h, xs, ys, B, B == 1, st);
            launch_cast_f2d(ys, y, (int64_t)B * N, st);
        }
    }
    // Z_j = P^{-1} V_j
    void apply_prec(int j) {
        if (v32) {
            precond_apply<float>(h, Vi32(j), (float*)Z + (int64_t)j * B * N, B, B == 1, st);
        } else if (!z32) {
            precond_apply<double>(h, Vi(j), (double*)Z + (int64_t)j * B * N, B, B == 1, st);
        } else {
            launch_cast_d2f(Vi(j), v32buf, (int64_t)B * N, st);
            precond_apply<float>(h, v32buf, (float*)Z + (int64_t)j * B * N, B, B == 1, st);
        }
    }
    // w = K Z_j (in w32 when v32)
    void apply_op_z(int j) {
        if (!z32) {
            kkt_apply<double>(h, (double*)Z + (int64_t)j * B * N, w, B, B == 1, st);
        } else if (!op32) {
            launch_cast_f2d((float*)Z + (int64_t)j * B * N, zt, (int64_t)B * N, st);
            kkt_apply<double>(h, zt, w, B, B == 1, st);
        } else if (v32) {
            kkt_apply<float>(h, (float*)Z + (int64_t)j * B * N, w32, B, B == 1, st);
        } else {
            kkt_apply<float>(h, (float*)Z + (int64_t)j * B * N, w32, B, B == 1, st);
            launch_cast_f2d(w32, w, (int64_t)B * N, st);
        }
    }
    // V_0 = r / ||r|| per member (kd.nrm holds ||r||^2; the cycle-start kernel
    // leaves 1/||r|| there)
    void start_basis(const double* r) {
        if (v32)
            launch_copy_scale_rows<float>(r, Vi32(0), kd.nrm, N, B, N, st);
        else
            launch_copy_scale_rows<double>(r, Vi(0), kd.nrm, N, B, N, st);
    }
    void dcgs_dots(int nv, bool with_w) {
        if (v32)
            launch_dcgs_dots<float>((const float*)V, vs, nv, with_w ? w32 : nullptr, N, B, N, kd.active, kd.pending,
                                    partial, nblk, st);
        else
            launch_dcgs_dots<double>((const double*)V, vs, nv, with_w ? w : nullptr, N, B, N, kd.active, kd.pending,
                                     partial, nblk, st);
    }
    void dcgs_update(int nv) {
        if (v32)
            launch_dcgs_update<float>((float*)V, vs, nv, w32, N, B, N, kd.coef, kd.scal, kd.active, nblk, st);
        else
            launch_dcgs_update<double>((double*)V, vs, nv, w, N, B, N, kd.coef, kd.scal, kd.active, nblk, st);
    }
    // bytes per element of the basis
    double vbytes() const { return v32 ? 4.0 : 8.0; }
    // per-member squared norms of x (FP64) -> host
    void norms2(const double* x, std::vector<double>& out) {
        launch_norm(x, N, B, N, partial, nblk, st);
        launch_reduce_partials(partial, nblk, 1, B, kd.nrm, 1, 0, st);
        readback(kd.nrm, out);
    }
    void readback(const double* d, std::vector<double>& out) {
        out.resize(B);
        SG_HIP(hipMemcpyAsync(h.h_pinned, d, sizeof(double) * B, hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
        std::memcpy(out.data(), h.h_pinned, sizeof(double) * B);
    }
    // r = b - K x, returns squared norms (r left in `r`)
    void residual(const double* b, const double* x, double* r, bool fp32, std::vector<double>& nr2) {
        apply_op(x, r, fp32);
        launch_sub_norm(b, r, N, B, N, partial, nblk, st);
        launch_reduce_partials(partial, nblk, 1, B, kd.nrm, 1, 0, st);
        readback(kd.nrm, nr2);
    }
};

// Restarted FGMRES on K x = b from the current x for the members with
// todo[b] != 0.  Member b stops when ||b - K x|| <= tol_abs[b] (true residual,
// checked at the start of each cycle) or when its own iteration count reaches
// max_iter; with max_cycles > 0 at most that many cycles run (the inner
// solves of iterative refinement run one cycle and stop on the Arnoldi
// estimate).  All stopping decisions are per member, so a member's arithmetic
// never depends on the other members of the batch.
//
// Inside a cycle the decisions are taken on the device: after each iteration
// k_conv_check clears a member's flag once its estimate reaches its tolerance
// or its iteration limit, and every later launch of the operator, the
// preconditioner and the Arnoldi passes skips that member.  The host reads the
// flags back only every few iterations (fewer when the estimates' recent
// reduction rate predicts convergence is still far off), and stops launching
// once no member is left.
//
// boundary (optional) runs after each cycle-start decision; when it returns
// true it has changed members' right-hand sides or iterates (refilled slots),
// and the residual is formed again before the cycle starts.
void fgmres(Krylov& K, const double* b, double* x, const std::vector<double>& tol_abs, std::vector<int>& todo,
            bool fp32, int max_iter, int max_cycles, std::vector<double>& res_out, std::vector<int>& member_iters,
            std::vector<double>& member_bytes, int verbose, const std::function<bool()>& boundary = nullptr) {
    Handle& h = K.h;
    const int B = K.B, m = K.m;
    const int64_t N = K.N;
    hipStream_t st = K.st;
    double* r = h.ws.get_t<double>("kr", (size_t)B * N);
    std::vector<double> nr2, resid;
    std::vector<int> active(B, 0);
    // host copy of the device's per-member `pending` flags (DCGS2): set for the
    // members that ran an iteration, so their last Hessenberg column is
    // completed by the next dot pass; only used to count the members each
    // profiled pass really processes (profiling reads the flags back after
    // every iteration)
    std::vector<int> pend(B, 0);
    res_out.assign(B, 0.0);
    // pinned staging: [0, 2048) readbacks (double), [2048, 4096) tolerances,
    // ints from 4096: control upload [4][B]; ints from 8192: control readback [2][B]
    double* tol_up = h.h_pinned + 2048;
    int* ctl_up = reinterpret_cast<int*>(h.h_pinned + 4096);
    int* ctl_dn = reinterpret_cast<int*>(h.h_pinned + 8192);
    const bool profiling = h.prof.kind != SG_PROF_NONE;
    // bytes model: the operator and preconditioner on their storage types, the
    // Arnoldi passes on the basis storage
    const double s_op = K.op32 ? 4.0 : 8.0, s_pc = K.z32 ? 4.0 : 8.0, s_v = K.vbytes();
    const double it_bytes = model_operator_bytes(h, s_op) + model_precond_bytes(h, s_pc);
    const double res_bytes = model_operator_bytes(h, fp32 && K.op32 ? 4.0 : 8.0) + 3.0 * 8.0 * N;
    std::vector<int> it_start(B, 0);
    for (int cycle = 0; max_cycles <= 0 || cycle < max_cycles;) {
        K.residual(b, x, r, fp32, nr2);       // synchronises the stream
        for (int q = 0; q < B; ++q)
            if (todo[q]) member_bytes[q] += res_bytes;
        bool any = false;
        for (int q = 0; q < B; ++q) {
            res_out[q] = std::sqrt(nr2[q]);
            if (todo[q] && (res_out[q] <= tol_abs[q] || member_iters[q] >= max_iter)) todo[q] = 0;
            any = any || todo[q];
        }
        if (verbose)
            for (int q = 0; q < B; ++q)
                std::fprintf(stderr, "[sg] member %d iters %d true residual %.3e (tol %.3e)%s\n", q, member_iters[q],
                             res_out[q], tol_abs[q], fp32 ? " [fp32 inner]" : "");
        if (boundary && boundary()) continue;
        if (!any) break;
        ++cycle;
        for (int q = 0; q < B; ++q) it_start[q] = member_iters[q];
        // cycle start: g = (beta, 0, ...), V_0 = r / beta; the control block
        // (flags, iteration counts, limits, cycle lengths) and the tolerances
        for (int q = 0; q < B; ++q) {
            active[q] = todo[q];
            pend[q] = 0;
            ctl_up[q] = active[q];
            ctl_up[B + q] = member_iters[q];
            ctl_up[2 * B + q] = max_iter;
            ctl_up[3 * B + q] = 0;
            tol_up[q] = tol_abs[q];
        }
        SG_HIP(hipMemcpyAsync(K.ctl, ctl_up, sizeof(int) * 4 * B, hipMemcpyHostToDevice, st));
        SG_HIP(hipMemcpyAsync((void*)K.kd.tol, tol_up, sizeof(double) * B, hipMemcpyHostToDevice, st));
        launch_cycle_start(K.kd, m, K.kd.nrm, B, st);    // kd.nrm holds ||r||^2 from residual()
        K.start_basis(r);
        const bool dcgs = h.opt.arnoldi == SG_ARNOLDI_DCGS2;
        const int64_t vs = K.vs;
        // one FGMRES iteration: preconditioner, KKT apply, Arnoldi, Givens, stop test
        auto iteration = [&](int j) {
            h.active = K.kd.active;
            K.apply_prec(j);
            K.apply_op_z(j);
            h.active = nullptr;
            if (dcgs) {
                // DCGS2: the basis slots hold the candidates U (V = U R^{-1}); one
                // read-only pass gives the reorthogonalisation of u_j and the
                // projections of w, one update pass writes the next candidate u_{j+1}
                // members each pass processes (the kernels skip the others):
                // the dot pass those active or with a pending column, the update
                // pass the active ones
                int n_dots = 0, n_upd = 0;
                for (int q = 0; q < B; ++q) {
                    n_dots += (active[q] || pend[q]) ? 1 : 0;
                    n_upd += active[q] ? 1 : 0;
                }
                bool tp = prof_begin(h, SG_PROF_MULTIDOT, st);
                K.dcgs_dots(j, true);
                if (tp) prof_end(h, st, K.vbytes() * (j + 2) * (double)n_dots * N);
                launch_reduce_partials(K.partial, K.nblk, 2 * j + 3, B, K.kd.dots, kSlots, 0, st);
                launch_dcgs_finish(K.kd, m, j, 0, B, st);
                tp = prof_begin(h, SG_PROF_ARNOLDI_UPD, st);
                K.dcgs_update(j);
                if (tp) prof_end(h, st, K.vbytes() * (j + 3) * (double)n_upd * N);   // read U_0..U_j and w, write u_{j+1}
                for (int q = 0; q < B; ++q) pend[q] = active[q];
            } else {
                const int nv = j + 1;
                // CGS2: h1 = V^T w; w1 = w - V h1; h2 = V^T w1; w2 = w1 - V h2
                const bool tp = prof_begin(h, SG_PROF_MULTIDOT, st);
                launch_multidot(K.Vi(0), vs, nv, K.w, N, B, N, K.partial, K.nblk, st);
                if (tp) prof_end(h, st, 8.0 * (nv + 1) * (double)B * N);
                launch_reduce_partials(K.partial, K.nblk, nv, B, K.kd.h1, m + 1, 0, st);
                launch_cgs_update_dot(K.Vi(0), vs, nv, K.kd.h1, m + 1, K.w, N, B, N, K.partial, K.nblk, st);
                launch_reduce_partials(K.partial, K.nblk, nv, B, K.kd.h2, m + 1, 0, st);
                launch_cgs_update_norm(K.Vi(0), vs, nv, K.kd.h2, m + 1, K.w, K.Vi(j + 1), N, B, N, K.partial,
                                       K.nblk, st);
                launch_reduce_partials(K.partial, K.nblk, 1, B, K.kd.nrm, 1, 0, st);
                launch_arnoldi_finish(K.kd, m, j, B, st);
                launch_scale_vec(K.Vi(j + 1), K.kd.nrm, 1, N, B, N, st);
            }
            launch_conv_check(K.kd, j, B, st);
        };
        const int zk = (K.z32 ? 1 : 0) + (K.op32 ? 2 : 0) + (K.v32 ? 4 : 0);
        // (capture needs a created stream; the legacy default stream cannot be captured)
        const bool graphs = h.opt.use_graphs && st != nullptr && !profiling && h.opt.cheb_steps <= 9;
        if (graphs && h.graphs.gen != h.ws.generation()) {
            h.graphs.clear();
            h.graphs.gen = h.ws.generation();
        }
        // host checks: the estimate and iteration of each active member at the
        // last check (the cycle start: the true residual)
        std::vector<double> est_prev(B), est(B);
        std::vector<int> it_prev(B, -1);
        for (int q = 0; q < B; ++q) est_prev[q] = res_out[q];
        int next_check = 0;
        int jlast = -1;
        for (int j = 0; j < m; ++j) {
            jlast = j;
            if (graphs && h.graphs.warm[zk]) {
                auto key = std::make_pair(j, zk);
                auto it = h.graphs.exec.find(key);
                if (it == h.graphs.exec.end()) {
                    hipGraph_t g = nullptr;
                    SG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                    try {
                        iteration(j);
                    } catch (...) {
                        h.active = nullptr;
                        (void)hipStreamEndCapture(st, &g);
                        if (g) (void)hipGraphDestroy(g);
                        throw;
                    }
                    SG_HIP(hipStreamEndCapture(st, &g));
                    hipGraphExec_t ex = nullptr;
                    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    SG_HIP(e);
                    it = h.graphs.exec.emplace(key, ex).first;
                }
                SG_HIP(hipGraphLaunch(it->second, st));
            } else {
                iteration(j);
            }
            if (!profiling && j < next_check && j < m - 1) continue;
            // read the flags, iteration counts and estimates back
            SG_HIP(hipMemcpyAsync(ctl_dn, K.ctl, sizeof(int) * 2 * B, hipMemcpyDeviceToHost, st));
            K.readback(K.kd.resid, resid);    // synchronises the stream
            bool still = false;
            int ahead = 8;                     // iterations until the next check
            for (int q = 0; q < B; ++q) {
                if (!active[q]) continue;
                member_iters[q] = ctl_dn[B + q];
                active[q] = ctl_dn[q];
                if (!active[q]) continue;
                still = true;
                // iterations the estimate still needs at its recent reduction rate
                const int done = j - it_prev[q];
                double need = 1.0;
                if (resid[q] > tol_abs[q] && resid[q] < est_prev[q] && done > 0) {
                    const double rate = std::log(resid[q] / est_prev[q]) / done;   // < 0
                    need = std::log(tol_abs[q] / resid[q]) / rate;
                }
                est_prev[q] = resid[q];
                it_prev[q] = j;
                ahead = std::min(ahead, std::max(1, (int)std::floor(0.8 * need)));
            }
            if (!still) break;
            next_check = j + ahead;
        }
        if (dcgs && jlast >= 0) {
            // reorthogonalise the last candidates (slot jlast + 1) of the members whose
            // last column is still pending, and commit that column
            K.dcgs_dots(jlast + 1, false);
            launch_reduce_partials(K.partial, K.nblk, jlast + 2, B, K.kd.dots, kSlots, 0, st);
            launch_dcgs_finish(K.kd, m, jlast + 1, 1, B, st);
        }
        launch_back_solve(K.kd, m, K.kd.jend, B, st);
        launch_multi_axpy(K.Z, K.z32 ? 1 : 0, (int64_t)B * N, m, K.kd.jend, K.kd.y, m, x, N, B, N, st);
        // iteration counts of the members still active at the last check
        SG_HIP(hipMemcpyAsync(ctl_dn, K.ctl, sizeof(int) * 2 * B, hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));     // the staging area is reused next cycle
        for (int q = 0; q < B; ++q)
            if (todo[q]) {
                member_iters[q] = ctl_dn[B + q];
                // k iterations: k (operator + preconditioner), the Arnoldi passes of
                // steps 0..k-1 (DCGS2: (j+2) + (j+3) vectors, CGS2 one more update
                // pass), the start vector and the cycle-end combination of k Z vectors
                const double k = member_iters[q] - it_start[q];
                const double arn = dcgs ? k * k + 4.0 * k : 1.5 * k * k + 6.5 * k;
                member_bytes[q] += k * it_bytes + s_v * N * arn + 2.0 * s_v * N + (k * s_pc + 16.0) * N;
            }
        if (graphs) {
            if (h.graphs.gen != h.ws.generation()) {   // buffers allocated in this cycle: recapture later
                h.graphs.clear();
                h.graphs.gen = h.ws.generation();
            }
            h.graphs.warm[zk] = true;
        }
    }
}

}  // namespace

int solve(Handle& h, const double* b_dev, double* x_dev, sg_solve_info* info, SlotFeed* feed) {
    using Clock = std::chrono::steady_clock;
    const auto t0 = Clock::now();
    const Shape& s = h.s;
    const int B = h.B;
    const int64_t N = 3 * s.blk;
    hipStream_t st = h.stream;
    // right-hand side with a zero boundary ring
    double* b = h.ws.get_t<double>("sb", (size_t)B * N);
    SG_HIP(hipMemcpyAsync(b, b_dev ? b_dev : h.d_rhs, sizeof(double) * B * N, hipMemcpyDeviceToDevice, st));
    launch_zero_ring<double>(b, s.n, (int64_t)B * 3 * s.nt * s.nxi, st);
    launch_fill_zero<double>(x_dev, (int64_t)B * N, st);

    const bool fp32 = h.opt.precision == SG_PREC_FP32_REFINE;
    const bool pc32 = h.opt.precision == SG_PREC_FP32_PRECOND;
    h.prof.kind = h.opt.profile;
    h.prof.reset();
    Krylov K(h, fp32 || pc32, fp32, fp32 && h.opt.basis_fp32 != 0);
    std::vector<double> bn2;
    K.norms2(b, bn2);
    std::vector<double> tol(B), res(B, 0.0);
    std::vector<int> todo(B, 1);
    for (int q = 0; q < B; ++q) tol[q] = h.opt.rtol * std::sqrt(bn2[q]);
    std::vector<int> member_iters(B, 0), member_outer(B, 0);
    std::vector<double> member_bytes(B, 0.0);   // model of the algorithmic HBM bytes per member
    std::vector<Clock::time_point> t_start(B, t0);
    std::vector<int> live(B, 1);    // slot holds a problem whose solve has not been reported (feed)

    auto report = [&](int q, double ms) {
        sg_solve_info r{};
        const double bn = std::sqrt(bn2[q]);
        const double rel = bn > 0 ? res[q] / bn : 0.0;
        const bool conv = rel <= h.opt.rtol;
        r.iters = member_iters[q];
        r.outer_refinements = member_outer[q];
        r.converged = conv ? 1 : 0;
        r.status = conv ? SG_OK : SG_NOT_CONVERGED;
        r.rel_res_true = rel;
        r.t_setup_ms = h.t_setup_ms;
        r.t_solve_ms = ms;
        r.latency_ms = ms;
        r.bytes_moved = member_bytes[q];
        return r;
    };
    // restart boundary with a feed: report the members whose solve ended,
    // then load new problems into the free slots (x = 0, their own b)
    auto boundary = [&]() -> bool {
        if (!feed) return false;
        const auto now = Clock::now();
        for (int q = 0; q < B; ++q)
            if (live[q] && !todo[q]) {
                feed->done(q, x_dev + q * N,
                           report(q, std::chrono::duration<double, std::milli>(now - t_start[q]).count()), st);
                live[q] = 0;
            }
        bool refilled = false;
        for (int q = 0; q < B; ++q) {
            if (live[q]) continue;
            sg_problem p{};
            if (!feed->next(q, p)) continue;
            set_member(h, q, p);
            SG_HIP(hipMemcpyAsync(b + q * N, h.d_rhs + q * N, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
            launch_zero_ring<double>(b + q * N, s.n, (int64_t)3 * s.nt * s.nxi, st);
            launch_fill_zero<double>(x_dev + q * N, N, st);
            live[q] = 1;
            todo[q] = 1;
            member_iters[q] = 0;
            member_outer[q] = 0;
            member_bytes[q] = 0.0;
            t_start[q] = Clock::now();
            refilled = true;
        }
        if (refilled) {
            K.norms2(b, bn2);
            for (int q = 0; q < B; ++q)
                if (todo[q]) tol[q] = h.opt.rtol * std::sqrt(bn2[q]);
        }
        return refilled;
    };

    if (!fp32) {
        fgmres(K, b, x_dev, tol, todo, false, h.opt.max_iter, 0, res, member_iters, member_bytes, h.opt.verbose,
               boundary);
    } else {
        // FP64 iterative refinement: r = b - K64 x (FP64 storage and sums);
        // one inner FGMRES cycle on K d = r with the operator and the
        // preconditioner on FP32 storage (the operator's stiffness sums in
        // FP64, so its products are accurate to FP32 rounding of the stored
        // vectors) and the Arnoldi basis in FP32 storage with FP64 sums
        // (basis_fp32), stopping on its estimate at inner_rtol ||r||; x += d
        // in FP64.  Every decision is per member (batch invariant).
        double* r = h.ws.get_t<double>("sr", (size_t)B * N);
        double* d = h.ws.get_t<double>("sd", (size_t)B * N);
        std::vector<double> nr2;
        const double res_bytes = model_operator_bytes(h, 8.0) + 3.0 * 8.0 * N;
        while (true) {
            K.residual(b, x_dev, r, false, nr2);
            for (int q = 0; q < B; ++q) {
                if (todo[q]) member_bytes[q] += res_bytes;
                res[q] = std::sqrt(nr2[q]);
                if (todo[q] && (res[q] <= tol[q] || member_iters[q] >= h.opt.max_iter)) todo[q] = 0;
            }
            if (boundary()) continue;
            std::vector<int> todo32(B, 0);
            std::vector<double> tol_in(B, 0.0);
            bool any = false;
            for (int q = 0; q < B; ++q) {
                if (!todo[q]) continue;
                tol_in[q] = std::max(h.opt.inner_rtol * res[q], 0.5 * tol[q]);
                ++member_outer[q];
                todo32[q] = 1;
                any = true;
            }
            if (!any) break;
            launch_fill_zero<double>(d, (int64_t)B * N, st);
            std::vector<double> rin;
            fgmres(K, r, d, tol_in, todo32, true, h.opt.max_iter, 1, rin, member_iters, member_bytes, h.opt.verbose);
            launch_axpby(1.0, d, 1.0, x_dev, (int64_t)B * N, st);
            for (int q = 0; q < B; ++q)
                if (todo32[q]) member_bytes[q] += 3.0 * 8.0 * N;   // x += d
        }
    }
    SG_HIP(hipStreamSynchronize(st));
    const auto t1 = Clock::now();
    const double pms = prof_collect_ms(h);
    h.prof.kind = SG_PROF_NONE;     // only sg_solve is profiled
    bool all = true;
    for (int q = 0; q < B; ++q) {
        const sg_solve_info r = report(q, std::chrono::duration<double, std::milli>(t1 - t_start[q]).count());
        if (live[q]) all = all && r.converged;
        if (info) {
            info[q] = r;
            info[q].prof_ms = pms;
            info[q].prof_bytes = h.prof.bytes;
            info[q].prof_launches = (int32_t)h.prof.used;
        }
    }
    return all ? SG_OK : SG_NOT_CONVERGED;
}

}  // namespace sg
