// Element-sweep kernels for the stochastic-Galerkin operator on gfx950.
//
// The SG operator Y_j = sum_k K_k W_{k,j} (W_{0,j} = X_j, W_{k,j} =
// g- X_{j-e_k} + g+ X_{j+e_k}) is evaluated element by element:
//   K_k = sum_e c_{k,e} K_ref,  so  (sum_k K_k W_k)|_e = K_ref (sum_k c_{k,e} W_k|_e),
// i.e. the chaos neighbours are combined at the four corners of each element
// with that element's coefficients, and one reference-element stiffness
// (1/6)[4 -1 -2 -1; ...] is applied per element and output column.  For local
// corner a with opposite corner o and corner sum s this is (5 v_a - v_o - s)/6.
//
// Work mapping (64-wide wavefronts): a wavefront owns one output chaos column
// j; its two 32-lane halves each walk a strip of RS node rows (2, 4 or 8,
// chosen per shape by the autotuner) of a 30-column x-tile.  Lane l holds node
// column X = 30*tx + l - 1 (lanes 0 and 31 are halos), loads each input value
// once per row, gets the x+1 neighbour by a lane shuffle and keeps the previous
// row in registers, so every input value is read about once per output
// column.  The node value is the sum of the corner contributions of its four
// elements: two from its own lane (this and the previous element row) and two
// from the lane to the left.  Blocks (4 wavefronts = 4 consecutive output
// columns of one spatial tile) are numbered so that each XCD receives a
// contiguous range of tiles with all their chaos columns: the neighbour columns
// a tile reads stay in that XCD's L2.  Each neighbour column is loaded once per
// output column that needs it; the strips are limited by load latency more
// than by bandwidth, so in the solve path the next chaos term's loads are kept
// in flight while the current term is accumulated (sg_strip).
#include "common.hpp"

// No automatic contraction in this file: every fused multiply-add is written
// out (fmadd), so each kernel's rounding sequence is the one in the source and
// the strip variants give bit-identical results whatever the code around the
// arithmetic looks like after inlining.
#pragma clang fp contract(off)

namespace sg {

namespace {

constexpr int GW = 32;          // lanes per strip group
constexpr int GOUT = GW - 2;    // output node columns per group
constexpr int KMAX = 8;         // modes handled by the sweep kernels

__device__ __forceinline__ int xcd_swizzle(int bid, int nb_padded) {
    const int per = nb_padded >> 3;
    return (bid & 7) * per + (bid >> 3);
}

template <typename T>
__device__ __forceinline__ T shdn(T v) {
    return __shfl_down(v, 1, GW);
}
template <typename T>
__device__ __forceinline__ T shup(T v) {
    return __shfl_up(v, 1, GW);
}

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Reference-element stiffness on a corner vector: k_a = (5 v_a - v_opp - s)/6.
__device__ __forceinline__ void kref(double v0, double v1, double v2, double v3, double& k0, double& k1, double& k2,
                                     double& k3) {
    const double s = (v0 + v1) + (v2 + v3);
    const double sixth = 1.0 / 6.0;
    k0 = (fmadd(5.0, v0, -v2) - s) * sixth;
    k1 = (fmadd(5.0, v1, -v3) - s) * sixth;
    k2 = (fmadd(5.0, v2, -v0) - s) * sixth;
    k3 = (fmadd(5.0, v3, -v1) - s) * sixth;
}

struct SweepGeom {
    int tiles_x, tiles_y, nchunks, nb;
};

// Occupancy hints per strip height (registers grow with the rows per strip).
constexpr int sweep_waves(int rs, int bytes, bool two) {
    return two ? (rs <= 2 ? 5 : rs <= 4 ? 3 : 2) : (rs <= 2 ? 6 : rs <= 4 ? 4 : bytes == 8 ? 2 : 3);
}
constexpr int kkt_waves(int rs, int bytes) { return rs <= 2 ? 4 : rs <= 4 ? 3 : 2; }

// One term of the SG sum at output column j: mean (k = -1: c0 X_j) or mode
// k+1 (c_{k+1,e} (g- F_{j-e_k} + g+ F_{j+e_k}), restricted to lower/upper).
// A term with a single input column holds it in the first slot (ia, ga).
struct Term {
    int ia, ib;
    double ga, gb;
    int k;
};

__device__ __forceinline__ bool term_at(int k, int j, int M, const int32_t* __restrict__ nidx,
                                        const double* __restrict__ nval, uint32_t mask, bool lower, bool upper,
                                        Term& t) {
    t.k = k;
    if (k < 0) {
        t.ia = j;
        t.ib = -1;
        t.ga = 1.0;
        t.gb = 0.0;
        return true;
    }
    if (!((mask >> k) & 1u)) return false;
    const int base = (j * M + k) * 2;
    t.ia = lower ? nidx[base] : -1;
    t.ib = upper ? nidx[base + 1] : -1;
    t.ga = nval[base];
    t.gb = nval[base + 1];
    if (t.ia < 0) {             // a term with one input column keeps it in the first slot
        t.ia = t.ib;
        t.ga = t.gb;
        t.ib = -1;
    }
    return t.ia >= 0;
}

__device__ __forceinline__ int next_term(int k, int j, int M, const int32_t* __restrict__ nidx,
                                         const double* __restrict__ nval, uint32_t mask, bool lower, bool upper,
                                         Term& t) {
    for (; k < M; ++k)
        if (term_at(k, j, M, nidx, nval, mask, lower, upper, t)) return k;
    return M;
}

// Row-strip helpers for strips of RS node rows per 32-lane group (RS is a
// launch parameter chosen per shape by the autotuner; every choice sums the
// same terms per node in the same order).
template <int RS>
struct Sweep {
    static constexpr int ER = 2 * RS + 1;   // element rows of a block's tile (both strips)

    // Coefficient modes 1..M of the block's element tile (element rows
    // ybase-1 .. ybase+2RS-1, element columns of the 32 lanes), zero off the
    // grid, into LDS as [mode-1][row][lane]: the block's four wavefronts then
    // read them from LDS instead of through the vector memory path.
    static __device__ __forceinline__ void stage_coef(double* sc, const double* __restrict__ coef, int64_t cplane, int M, int n,
                                                      int tx, int ty) {
        const int ybase = ty * 2 * RS;
        const int total = M * ER * GW;
        // every load first (clamped addresses), then the masked LDS stores: a
        // masked load per store would cost one memory latency each
        constexpr int NQ = (KMAX * ER * GW + 255) / 256;
        double tmp[NQ];
    #pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int q = min((int)threadIdx.x + 256 * i, total - 1);
            const int ln = q % GW, r = (q / GW) % ER, k = q / (GW * ER);
            const int X = min(max(tx * GOUT + ln - 1, 0), n - 1);
            const int ey = min(max(ybase - 1 + r, 0), n - 1);
            tmp[i] = coef[(int64_t)(k + 1) * cplane + (int64_t)ey * n + X];
        }
    #pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int q = threadIdx.x + 256 * i;
            if (q < total) {
                const int ln = q % GW, r = (q / GW) % ER;
                const int X = tx * GOUT + ln - 1;
                const int ey = ybase - 1 + r;
                const bool ok = X >= 0 && X <= n - 1 && ey >= 0 && ey <= n - 1;
                sc[q] = ok ? tmp[i] : 0.0;
            }
        }
    }
    // Per-lane strip geometry: node rows y0-1 .. y0+RS (RS+2 rows) and element
    // rows y0-1 .. y0+RS-1 (RS+1 rows) of node column X.  Offsets are clamped into
    // the grid so that every load is in bounds; the masks zero what lies on the
    // Dirichlet ring or outside the grid.
    struct Strip {
        int n, xc, xe, y0;
        uint32_t nmask, emask;
        __device__ __forceinline__ void init(int n_, int X, int y0_) {
            n = n_;
            y0 = y0_;
            xc = min(max(X, 0), n);
            xe = min(max(X, 0), n - 1);
            const bool xin = X >= 1 && X <= n - 1;
            const bool xev = X >= 0 && X <= n - 1;
            nmask = 0;
            emask = 0;
    #pragma unroll
            for (int r = 0; r < RS + 2; ++r) {
                const int Y = y0 - 1 + r;
                if (xin && Y >= 1 && Y <= n - 1) nmask |= 1u << r;
            }
    #pragma unroll
            for (int r = 0; r < RS + 1; ++r) {
                const int ey = y0 - 1 + r;
                if (xev && ey >= 0 && ey <= n - 1) emask |= 1u << r;
            }
        }
        __device__ __forceinline__ int noff(int r) const { return min(max(y0 - 1 + r, 0), n) * (n + 1) + xc; }
        __device__ __forceinline__ int eoff(int r) const { return min(max(y0 - 1 + r, 0), n - 1) * n + xe; }
    };

    // v[r] += c_r * (corner values of element row r) for one input column stream
    // (vals = node values of the column at the RS+2 strip rows, already scaled).
    static __device__ __forceinline__ void corner_accumulate(double (&v)[RS + 1][4], const double (&vals)[RS + 2],
                                                             const double (&c)[RS + 1]) {
        double prev = vals[0];
        double prevR = shdn(prev);
    #pragma unroll
        for (int r = 0; r < RS + 1; ++r) {
            const double top = vals[r + 1];
            const double topR = shdn(top);
            v[r][0] = fmadd(c[r], prev, v[r][0]);
            v[r][1] = fmadd(c[r], prevR, v[r][1]);
            v[r][2] = fmadd(c[r], topR, v[r][2]);
            v[r][3] = fmadd(c[r], top, v[r][3]);
            prev = top;
            prevR = topR;
        }
    }

    template <typename T>
    static __device__ __forceinline__ void load_col(double (&vals)[RS + 2], const T* __restrict__ col, const Strip& st,
                                                    double g, bool accumulate) {
    #pragma unroll
        for (int r = 0; r < RS + 2; ++r) {
            double x = (double)col[st.noff(r)];
            x = ((st.nmask >> r) & 1u) ? x : 0.0;
            vals[r] = accumulate ? fmadd(g, x, vals[r]) : g * x;
        }
    }

    // Coefficients of term k on the strip's element rows (mean: c0; staged
    // tile in LDS when sc is set, else the coefficient planes), zero off the
    // grid.  The global path always loads (the mean term reads plane 0 and
    // discards it), so the number of loads in flight is the same for every
    // term.
    static __device__ __forceinline__ void load_coef(double (&c)[RS + 1], int k, const Strip& st, double c0,
                                                     const double* __restrict__ sc, int grp, int gl,
                                                     const double* __restrict__ coef, int64_t cplane) {
        if (sc) {
            if (k < 0) {
    #pragma unroll
                for (int r = 0; r < RS + 1; ++r) c[r] = ((st.emask >> r) & 1u) ? c0 : 0.0;
            } else {
                const double* ck = sc + (k * ER + grp * RS) * GW + gl;    // staged, zero off the grid
    #pragma unroll
                for (int r = 0; r < RS + 1; ++r) c[r] = ck[r * GW];
            }
        } else {
            // masks applied by multiplication (a select would let the compiler
            // branch around the load, and the branch join waits for every load)
            const double* ck = coef + (int64_t)(k + 1) * cplane;
            const double sm = k < 0 ? 0.0 : 1.0, sk = k < 0 ? 1.0 : 0.0;
    #pragma unroll
            for (int r = 0; r < RS + 1; ++r) {
                const double cv = ck[st.eoff(r)];
                const double mf = ((st.emask >> r) & 1u) ? 1.0 : 0.0;
                c[r] = (cv * sm + c0 * sk) * mf;
            }
        }
    }

    // Raw node values of a term's lower and upper input columns at the strip's
    // RS+2 rows.  They are combined (masked, scaled, then summed)
    // only when the term is accumulated, so that loads issued for the next term
    // stay in flight while the current term is computed.
    template <typename T>
    struct Raw {
        T a[RS + 2], b[RS + 2];
    };
    // TWO: terms may have two input columns (the second is then always loaded,
    // from the first column when absent, and selected away); without TWO every
    // term has exactly one.  Either way the loads per term are a fixed count.
    template <bool TWO, typename T>
    static __device__ __forceinline__ void load_raw(Raw<T>& R, const Term& t, const T* __restrict__ F,
                                                    int64_t nodes, const Strip& st) {
        const T* ca = F + (int64_t)t.ia * nodes;       // every term has its first column
    #pragma unroll
        for (int r = 0; r < RS + 2; ++r) R.a[r] = ca[st.noff(r)];
        if (TWO) {
            const T* cb = F + (int64_t)(t.ib >= 0 ? t.ib : t.ia) * nodes;
    #pragma unroll
            for (int r = 0; r < RS + 2; ++r) R.b[r] = cb[st.noff(r)];
        }
    }
    // value of the term at strip row r (masked, scaled, then summed)
    template <bool TWO, typename T>
    static __device__ __forceinline__ double combine_row(const Raw<T>& R, const Term& t, const Strip& st, int r) {
        const bool in = (st.nmask >> r) & 1u;
        double val = t.ga * (in ? (double)R.a[r] : 0.0);
        if (TWO) {
            const double v2 = fmadd(t.gb, in ? (double)R.b[r] : 0.0, val);
            val = t.ib >= 0 ? v2 : val;
        }
        return val;
    }
    // corner_accumulate of one term, its row values combined on the fly
    template <bool TWO, typename T>
    static __device__ __forceinline__ void accumulate_term(double (&v)[RS + 1][4], const Raw<T>& R, const Term& t,
                                                           const Strip& st, const double (&c)[RS + 1]) {
        double prev = combine_row<TWO>(R, t, st, 0);
        double prevR = shdn(prev);
    #pragma unroll
        for (int r = 0; r < RS + 1; ++r) {
            const double top = combine_row<TWO>(R, t, st, r + 1);
            const double topR = shdn(top);
            v[r][0] = fmadd(c[r], prev, v[r][0]);
            v[r][1] = fmadd(c[r], prevR, v[r][1]);
            v[r][2] = fmadd(c[r], topR, v[r][2]);
            v[r][3] = fmadd(c[r], top, v[r][3]);
            prev = top;
            prevR = topR;
        }
    }

    // Corner vectors v[r][.] of element rows y0-1+r of the SG operator applied to
    // field F at output column j: c0 X_j (mean, if with_mean) plus, for every
    // mode k in mask, c_{k,e} (g- F_{j-e_k} [lower] + g+ F_{j+e_k} [upper]).
    // The next term's raw node values are loaded into a second buffer while
    // the current term is accumulated, and moved into the first afterwards.
    // The current term's coefficients are loaded before the next term's
    // values (loads complete in order, so the wait for them leaves the next
    // term's loads in flight), the present modes are a bit set found before
    // any vector load, and a scheduling barrier keeps the loads ahead of the
    // arithmetic.  The per-node arithmetic is the same for every strip height.
    template <bool TWO, typename T>
    static __device__ __forceinline__ void sg_strip(double (&v)[RS + 1][4], const Strip& st, const T* __restrict__ F,
                                                    int64_t nodes, int j, int M, const int32_t* __restrict__ nidx,
                                                    const double* __restrict__ nval, uint32_t mask, bool lower,
                                                    bool upper, bool with_mean, double c0,
                                                    const double* __restrict__ sc, int grp, int gl,
                                                    const double* __restrict__ coef, int64_t cplane) {
        double c[RS + 1];
        Raw<T> RA, RB;                                 // current and next term's raw node values
        Term tA, tB;
        // the present modes as a bit set (one scalar pass before any vector
        // load), so that no loop separates a term's loads from their use
        uint32_t todo = 0;
        for (int k = 0; k < M; ++k) {
            Term t;
            if (term_at(k, j, M, nidx, nval, mask, lower, upper, t)) todo |= 1u << k;
        }
        auto pop = [&](Term& t) -> int {
            if (!todo) return M;
            const int k = __builtin_ctz(todo);
            todo &= todo - 1u;
            term_at(k, j, M, nidx, nval, mask, lower, upper, t);
            return k;
        };
        int kA = M;
        if (with_mean) {
            kA = -1;
            term_at(-1, j, M, nidx, nval, mask, lower, upper, tA);
        } else {
            kA = pop(tA);
        }
        if (kA >= M) return;
        load_raw<TWO>(RA, tA, F, nodes, st);
        // each iteration decides whether a next term exists before issuing any
        // load, so its loads and arithmetic are straight-line code; the copy of
        // the next term's raw values comes after the current term's arithmetic
    #pragma unroll 1
        while (true) {
            const int kB = pop(tB);
            if (kB >= M) break;                        // A is the last term
            load_coef(c, kA, st, c0, sc, grp, gl, coef, cplane);
            load_raw<TWO>(RB, tB, F, nodes, st);
            __builtin_amdgcn_sched_barrier(0);         // keep those loads ahead of the arithmetic
            accumulate_term<TWO>(v, RA, tA, st, c);
            __builtin_amdgcn_sched_barrier(0);
            RA = RB;
            tA = tB;
            kA = kB;
        }
        load_coef(c, kA, st, c0, sc, grp, gl, coef, cplane);
        accumulate_term<TWO>(v, RA, tA, st, c);
    }

    // The same sums without load pipelining: each term's node values are
    // combined as they arrive (the next term's loads are issued before the
    // current term is accumulated, but the compiler waits for them within the
    // iteration).  Lighter on registers; used by the standalone SG apply, where
    // it measured faster than the pipelined strip at the occupancy it allows.
    template <typename T>
    static __device__ __forceinline__ void load_term(double (&vals)[RS + 2], const Term& t, const T* __restrict__ F,
                                                     int64_t nodes, const Strip& st) {
        load_col(vals, F + (int64_t)t.ia * nodes, st, t.ga, false);
        if (t.ib >= 0) load_col(vals, F + (int64_t)t.ib * nodes, st, t.gb, true);
    }
    template <typename T>
    static __device__ __forceinline__ void sg_strip_direct(double (&v)[RS + 1][4], const Strip& st, const T* __restrict__ F,
                                                           int64_t nodes, int j, int M, const int32_t* __restrict__ nidx,
                                                           const double* __restrict__ nval, uint32_t mask, bool lower,
                                                           bool upper, bool with_mean, double c0,
                                                           const double* __restrict__ sc, int grp, int gl,
                                                           const double* __restrict__ coef, int64_t cplane) {
        double vals[RS + 2], nvals[RS + 2];
        double c[RS + 1];
        Term cur, nxt;
        int k = next_term(with_mean ? -1 : 0, j, M, nidx, nval, mask, lower, upper, cur);
        if (k >= M) return;
        load_term(vals, cur, F, nodes, st);
    #pragma unroll 1
        while (true) {
            const int kn = next_term(k + 1, j, M, nidx, nval, mask, lower, upper, nxt);
            const bool more = kn < M;
            if (more) load_term(nvals, nxt, F, nodes, st);
            load_coef(c, k, st, c0, sc, grp, gl, coef, cplane);
            corner_accumulate(v, vals, c);
            if (!more) break;
    #pragma unroll
            for (int r = 0; r < RS + 2; ++r) vals[r] = nvals[r];
            cur = nxt;
            k = kn;
        }
    }

    // Reference-element mass (h^2/36)[4 2 1 2; 2 4 2 1; 1 2 4 2; 2 1 2 4] on a
    // corner vector: m_a = w (2 s + 2 v_a - v_opp), w = h^2/36.
    static __device__ __forceinline__ void mass_accumulate(double (&e)[RS + 1][4], const double (&vals)[RS + 2],
                                                           const Strip& st, double w) {
        double prev = vals[0];
        double prevR = shdn(prev);
    #pragma unroll
        for (int r = 0; r < RS + 1; ++r) {
            const double top = vals[r + 1];
            const double topR = shdn(top);
            const double c = ((st.emask >> r) & 1u) ? w : 0.0;
            const double s2 = 2.0 * ((prev + prevR) + (topR + top));
            e[r][0] = fmadd(c, fmadd(2.0, prev, s2) - topR, e[r][0]);
            e[r][1] = fmadd(c, fmadd(2.0, prevR, s2) - top, e[r][1]);
            e[r][2] = fmadd(c, fmadd(2.0, topR, s2) - prev, e[r][2]);
            e[r][3] = fmadd(c, fmadd(2.0, top, s2) - prevR, e[r][3]);
            prev = top;
            prevR = topR;
        }
    }

    // Corner sums of the SG stiffness strip -> element results scaled by -s.
    static __device__ __forceinline__ void stiff_to_element(double (&v)[RS + 1][4], double s) {
    #pragma unroll
        for (int r = 0; r < RS + 1; ++r) {
            double k0, k1, k2, k3;
            kref(v[r][0], v[r][1], v[r][2], v[r][3], k0, k1, k2, k3);
            v[r][0] = -s * k0;
            v[r][1] = -s * k1;
            v[r][2] = -s * k2;
            v[r][3] = -s * k3;
        }
    }

    // Node values from per-element results e[r][.] (element rows y0-1+r): node
    // (X, Y) sums corners 0 and 3 of its own lane's element rows r and r-1 and
    // corners 1 and 2 of the lane to the left; non-interior nodes get zero.
    template <typename T>
    static __device__ __forceinline__ void emit_nodes(const double (&e)[RS + 1][4], const Strip& st, int gl, int X, int n,
                                               T* __restrict__ out) {
        const bool xout = gl >= 1 && gl <= GOUT && X <= n;
    #pragma unroll
        for (int r = 1; r < RS + 1; ++r) {
            const double A = e[r][0] + e[r - 1][3];
            const double Bl = shup(e[r][1] + e[r - 1][2]);
            const int Y = st.y0 - 1 + r;
            if (xout && Y <= n) out[(int64_t)Y * (n + 1) + X] = (T)(((st.nmask >> r) & 1u) ? A + Bl : 0.0);
        }
    }

    static __device__ __forceinline__ void zero_strip(double (&v)[RS + 1][4]) {
    #pragma unroll
        for (int r = 0; r < RS + 1; ++r) v[r][0] = v[r][1] = v[r][2] = v[r][3] = 0.0;
    }

    // Fused KKT apply, one output chaos column per wavefront, three residual blocks
    // in turn.  With the SG stiffness A (mean included) and Q1 mass M:
    //   steady (eq. stoch-system):  R^Y = M Y H^gamma - A L,  R^U = beta M U + M L,  R^L = M U - A Y
    //   time (eq. KKT:stoch-time-dependent, backward Euler, D = diag(1/2, 1, .., 1, 1/2)):
    //     R^Y_t = tau D_t M_gamma Y_t - M L_t - tau A L_t + M L_{t+1}
    //     R^U_t = beta tau D_t M U_t + tau M L_t
    //     R^L_t = -M Y_t - tau A Y_t + M Y_{t-1} + tau M U_t
    // Each block is (mass of a combination of diagonal columns) - s (stiffness strip),
    // formed per element and assembled once.
};

// KIND 0: Y = A X (all modes, mean included) for nt*nvec slices.
// KIND 1: hGS right-hand side of degree level d:
//         out_j = base_j - off_scale * sum_{k in mask} K_k (g- V_{j-e_k} [lower] + g+ V_{j+e_k} [upper]).
template <typename T, int KIND, int RS, bool TWO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sweep_waves(RS, sizeof(T), TWO)))) void k_sgx(int n, int M, int nxi, int nt, int64_t nodes, OpDev op, SweepGeom g,
                                             const T* __restrict__ x, T* __restrict__ y, int j0lvl, int L,
                                             uint32_t mask, int lower, int upper, const T* __restrict__ base,
                                             ColMap bmap, ColMap vmap, ColMap omap) {
    const int lb = xcd_swizzle(blockIdx.x, gridDim.x);
    if (lb >= g.nb) return;
    const int chunk = lb % g.nchunks;
    const int rest = lb / g.nchunks;
    const int tiles = g.tiles_x * g.tiles_y;
    const int tile = rest % tiles;
    const int slice = rest / tiles;
    if (op.active && !op.active[slice / nt]) return;
    const int tx = tile % g.tiles_x, ty = tile / g.tiles_x;
    // wavefront index is uniform: keep it (and everything derived from it) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = chunk * 4 + wave;                  // output column index (in the level for KIND 1)
    const int ncols = KIND == 0 ? nxi : L;
    using S = Sweep<RS>;
    if (l >= ncols) return;                          // uniform per wavefront; no block barriers below
    const int j = KIND == 0 ? l : j0lvl + l;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (GW - 1);
    const int grp = lane / GW;
    const int X = tx * GOUT + gl - 1;
    const int y0 = (ty * 2 + grp) * RS;
    const int mem_i = slice / nt;
    const int t = slice % nt;
    const int mem = op.mem_shared ? 0 : mem_i;
    const T* F = KIND == 0 ? x + (int64_t)slice * nxi * nodes
                           : x + (int64_t)mem_i * vmap.mstride + (int64_t)t * vmap.tstride;
    typename S::Strip st;
    st.init(n, X, y0);
    double v[RS + 1][4];
#pragma unroll
    for (int r = 0; r < RS + 1; ++r) v[r][0] = v[r][1] = v[r][2] = v[r][3] = 0.0;
    if constexpr (KIND == 0)
        S::sg_strip_direct(v, st, F, nodes, j, M, op.nbr_idx, op.nbr_val, mask, true, true, true,
                           op.mem[mem].c0, (const double*)nullptr, grp, gl,
                           op.coef64 + (int64_t)mem * op.coef_mstride, (int64_t)n * n);
    else
        S::template sg_strip<TWO>(v, st, F, nodes, j, M, op.nbr_idx, op.nbr_val, mask, lower != 0, upper != 0, false,
                                  op.mem[mem].c0, (const double*)nullptr, grp, gl,
                                  op.coef64 + (int64_t)mem * op.coef_mstride, (int64_t)n * n);
    T* out;
    const T* bas = nullptr;
    double scale = 1.0;
    if (KIND == 0) {
        out = y + (int64_t)slice * nxi * nodes + (int64_t)j * nodes;
    } else {
        const int c = slice * L + l;
        out = y + omap.off(c);
        bas = base + bmap.off(c);
        scale = op.off_sign * op.mem[mem].off_scale;
    }
    const bool xout = gl >= 1 && gl <= GOUT && X <= n;
    double k2p, k3p;
    {
        double k0, k1;
        kref(v[0][0], v[0][1], v[0][2], v[0][3], k0, k1, k2p, k3p);
    }
#pragma unroll
    for (int r = 1; r < RS + 1; ++r) {
        double k0, k1, k2, k3;
        kref(v[r][0], v[r][1], v[r][2], v[r][3], k0, k1, k2, k3);
        const double A = k0 + k3p;
        const double Bl = shup(k1 + k2p);
        const int Y = y0 - 1 + r;                 // node row of this output
        if (xout && Y <= n) {
            const bool inter = (st.nmask >> r) & 1u;    // node (X, Y) is interior (strip row r)
            const int64_t q = (int64_t)Y * (n + 1) + X;
            double val = 0.0;
            if (KIND == 0) {
                if (inter) val = A + Bl;
            } else {
                if (inter) val = fmadd(-scale, A + Bl, (double)bas[q]);
            }
            out[q] = (T)val;
        }
        k2p = k2;
        k3p = k3;
    }
}

template <typename T, bool TIME, int RS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kkt_waves(RS, sizeof(T))))) void k_sgx_kkt(
    int n, int M, int nxi, int nt, int64_t nodes, OpDev op, SweepGeom g, const T* __restrict__ x,
    T* __restrict__ y) {
    const int lb = xcd_swizzle(blockIdx.x, gridDim.x);
    if (lb >= g.nb) return;
    const int chunk = lb % g.nchunks;
    const int rest = lb / g.nchunks;
    const int tiles = g.tiles_x * g.tiles_y;
    const int tile = rest % tiles;
    const int slice = rest / tiles;
    if (op.active && !op.active[slice / nt]) return;   // uniform per block, before the barrier below
    const int tx = tile % g.tiles_x, ty = tile / g.tiles_x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = chunk * 4 + wave;
    using S = Sweep<RS>;
    // the block's four output columns run two full stiffness strips each over
    // the same element tile: its coefficients are staged once in LDS
    __shared__ double sc[KMAX * S::ER * GW];
    {
        const int mem_b = op.mem_shared ? 0 : (slice / nt);
        S::stage_coef(sc, op.coef64 + (int64_t)mem_b * op.coef_mstride, (int64_t)n * n, M, n, tx, ty);
    }
    __syncthreads();
    if (j >= nxi) return;                            // uniform per wavefront; no block barriers below
    const int lane = threadIdx.x & 63;
    const int gl = lane & (GW - 1);
    const int grp = lane / GW;
    const int X = tx * GOUT + gl - 1;
    const int y0 = (ty * 2 + grp) * RS;
    const int vec = slice / nt;
    const int t = slice % nt;
    const int mem = op.mem_shared ? 0 : vec;
    const MemberDev md = op.mem[mem];
    const int64_t blk = (int64_t)nt * nxi * nodes;
    const int64_t tst = (int64_t)nxi * nodes;
    const int64_t cj = (int64_t)j * nodes;
    const T* Yt = x + (int64_t)vec * 3 * blk + t * tst;
    const T* Ut = Yt + blk;
    const T* Lt = Ut + blk;
    T* RY = y + (int64_t)vec * 3 * blk + t * tst + cj;
    T* RU = RY + blk;
    T* RL = RU + blk;
    const double hinv = 1.0 / (double)n;
    const double w = hinv * hinv / 36.0;
    const double tau = TIME ? md.tau : 1.0;
    const double Dt = (TIME && (t == 0 || t == nt - 1)) ? 0.5 : 1.0;
    const double hgj = j == 0 ? 1.0 : md.hg;
    const double beta = md.beta;
    const double c0 = md.c0;
    typename S::Strip st;
    st.init(n, X, y0);
    double v[RS + 1][4];
    double vals[RS + 2];
    // R^Y
    S::zero_strip(v);
    S::template sg_strip<true>(v, st, Lt, nodes, j, M, op.nbr_idx, op.nbr_val, 0xffffffffu, true, true, true, c0, sc,
                               grp, gl,
                (const double*)nullptr, 0);
    S::stiff_to_element(v, tau);
    S::load_col(vals, Yt + cj, st, tau * Dt * hgj, false);
    if (TIME) {
        S::load_col(vals, Lt + cj, st, -1.0, true);
        if (t + 1 < nt) S::load_col(vals, Lt + tst + cj, st, 1.0, true);
    }
    S::mass_accumulate(v, vals, st, w);
    S::emit_nodes(v, st, gl, X, n, RY);
    // R^L
    S::zero_strip(v);
    S::template sg_strip<true>(v, st, Yt, nodes, j, M, op.nbr_idx, op.nbr_val, 0xffffffffu, true, true, true, c0, sc,
                               grp, gl,
                (const double*)nullptr, 0);
    S::stiff_to_element(v, tau);
    S::load_col(vals, Ut + cj, st, tau, false);
    if (TIME) {
        S::load_col(vals, Yt + cj, st, -1.0, true);
        if (t > 0) S::load_col(vals, Yt - tst + cj, st, 1.0, true);
    }
    S::mass_accumulate(v, vals, st, w);
    S::emit_nodes(v, st, gl, X, n, RL);
    // R^U
    S::zero_strip(v);
    S::load_col(vals, Ut + cj, st, beta * tau * Dt, false);
    S::load_col(vals, Lt + cj, st, tau, true);
    S::mass_accumulate(v, vals, st, w);
    S::emit_nodes(v, st, gl, X, n, RU);
}

// ---------------------------------------------------------------------------
// SG apply on FP64 storage with two nodes per lane.
//
// Y_j = c0 X_j (stiffness of the mean) + sum_k sum_{s = -,+} g K_k X_{j +- e_k}
// per slice (vector, time step).  A lane owns a pair of neighbouring node
// columns (one 16-byte load per node row), a 32-lane half owns 62 output node
// columns and PR node rows, the two halves of a wavefront sit one above the
// other, and the four wavefronts of a block take output columns chunk*16 +
// wave + 4q, q < 4, over the same element tile, whose coefficient modes are
// staged once in LDS.  Each wavefront streams one input column per item (the
// mean term, then every present neighbour of each mode in mask) with the next
// column's loads in flight while the current one is accumulated at the
// element corners; the element results become node values once per output
// column (the reference stiffness k_a = (5 v_a - v_opp - s)/6, then the sum of
// the four elements at each node, the left one through a lane shift).  Input
// nodes on the boundary ring are masked to zero as they are read, output ring
// nodes are written as zero.
// ---------------------------------------------------------------------------
constexpr int PR = 4;            // node rows per 32-lane half
constexpr int PNC = 4;           // output columns per wavefront
constexpr int PGX = 62;          // output node columns per tile (two per lane, 31 lanes)
constexpr int PER = 2 * PR + 1;  // element rows of a tile
constexpr int PEC = 64;          // element columns staged per tile

typedef double pd2 __attribute__((ext_vector_type(2)));
typedef pd2 pd2u __attribute__((aligned(8)));   // node pairs start on any 8-byte boundary

// lane l <- lane l+1, and lane l <- lane l-1 (64-bit values, row shifts by DPP)
__device__ __forceinline__ double dpp_from_right(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_from_left(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

struct PairItem {
    int col, k, j;   // input column, mode (-1: mean), output column
    double g;
    bool last, valid;
};

__global__ __launch_bounds__(256) void k_sgx_pair(int n, int M, int nxi, int nt, int64_t nodes, OpDev op,
                                                  uint32_t mask, const double* __restrict__ x,
                                                  double* __restrict__ y, int tiles_x, int tiles_y, int nchunks,
                                                  int nb) {
    __shared__ double sc[KMAX * PER * PEC];
    const int lb = xcd_swizzle(blockIdx.x, gridDim.x);
    if (lb >= nb) return;
    const int chunk = lb % nchunks;
    const int rest = lb / nchunks;
    const int tile = rest % (tiles_x * tiles_y);
    const int slice = rest / (tiles_x * tiles_y);
    if (op.active && !op.active[slice / nt]) return;   // uniform per block, before the barrier below
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int mem = op.mem_shared ? 0 : slice / nt;
    const double* coef = op.coef64 + (int64_t)mem * op.coef_mstride;
    const double c0 = op.mem[mem].c0;
    const int ex0 = PGX * tx;            // first element column of the tile
    const int ey0 = ty * 2 * PR - 1;     // first element row
    {
        // modes 1..M of the tile, clamped to the grid (elements off the grid
        // meet only masked ring nodes, so their coefficients never count)
        const int total = M * PER * PEC;
        for (int q = threadIdx.x; q < total; q += 256) {
            const int ec = q % PEC, r = (q / PEC) % PER, k = q / (PEC * PER);
            const int ex = min(ex0 + ec, n - 1);
            const int ey = min(max(ey0 + r, 0), n - 1);
            sc[q] = coef[(int64_t)(k + 1) * n * n + (int64_t)ey * n + ex];
        }
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jbase = chunk * 4 * PNC + wave;
    if (jbase >= nxi) return;            // uniform per wavefront; no block barriers below
    const int lane = threadIdx.x & 63;
    const int gl = lane & 31;
    const int grp = lane >> 5;
    const int x0 = ex0 + 2 * gl;          // first node column of the lane's pair
    const int y0 = (2 * ty + grp) * PR;   // first output node row of the half
    const double* F = x + (int64_t)slice * nxi * nodes;
    double* Yo = y + (int64_t)slice * nxi * nodes;
    // per strip row: the pair's offset (rows clamped to the grid, pairs past the
    // row end clamped into the column) and the masks of interior input nodes
    int rowoff[PR + 2];
    bool ok0[PR + 2], ok1[PR + 2];
#pragma unroll
    for (int r = 0; r < PR + 2; ++r) {
        const int Yr = y0 - 1 + r;
        rowoff[r] = (int)min((int64_t)min(max(Yr, 0), n) * (n + 1) + x0, nodes - 2);
        const bool yin = Yr >= 1 && Yr <= n - 1;
        ok0[r] = yin && x0 >= 1 && x0 <= n - 1;
        ok1[r] = yin && x0 + 1 <= n - 1;
    }
    const double* scl = sc + (grp * PR) * PEC + 2 * gl;
    // the wavefront's items, generated in scalar registers
    int q = 0, jc = jbase;
    uint32_t todo = 0;
    auto present = [&](int j) -> uint32_t {
        uint32_t m = 0;
        for (int k = 0; k < M; ++k) {
            if (!((mask >> k) & 1u)) continue;
            const int b = (j * M + k) * 2;
            if (op.nbr_idx[b] >= 0) m |= 1u << (2 * k);
            if (op.nbr_idx[b + 1] >= 0) m |= 1u << (2 * k + 1);
        }
        return m;
    };
    auto next_item = [&]() -> PairItem {
        PairItem it;
        if (todo) {
            const int sl = __builtin_ctz(todo);
            todo &= todo - 1u;
            const int b = (jc * M + (sl >> 1)) * 2 + (sl & 1);
            it.col = op.nbr_idx[b];
            it.g = op.nbr_val[b];
            it.k = sl >> 1;
            it.j = jc;
            it.last = todo == 0;
            it.valid = true;
            return it;
        }
        ++q;
        jc = jbase + 4 * q;
        if (q >= PNC || jc >= nxi) {
            it.col = 0; it.g = 0.0; it.k = -1; it.j = -1; it.last = false; it.valid = false;
            return it;
        }
        todo = present(jc);
        it.col = jc; it.g = c0; it.k = -1; it.j = jc; it.last = todo == 0; it.valid = true;
        return it;
    };
    // element-corner sums [row][element of the pair][corner]
    double acc[PR + 1][2][4];
#pragma unroll
    for (int r = 0; r < PR + 1; ++r)
#pragma unroll
        for (int e = 0; e < 2; ++e) acc[r][e][0] = acc[r][e][1] = acc[r][e][2] = acc[r][e][3] = 0.0;
    auto load = [&](pd2 (&V)[PR + 2], int col) {
        const double* p = F + (int64_t)col * nodes;
#pragma unroll
        for (int r = 0; r < PR + 2; ++r) V[r] = *(const pd2u*)(p + rowoff[r]);
    };
    auto accumulate = [&](const pd2 (&V)[PR + 2], const PairItem& it) {
        const double g = it.g;
        double w0[PR + 2], w1[PR + 2], w2[PR + 2];
#pragma unroll
        for (int r = 0; r < PR + 2; ++r) {
            w0[r] = g * (ok0[r] ? V[r].x : 0.0);
            w1[r] = g * (ok1[r] ? V[r].y : 0.0);
            w2[r] = dpp_from_right(w0[r]);   // the right neighbour pair's first node
        }
        if (it.k < 0) {
#pragma unroll
            for (int r = 0; r < PR + 1; ++r) {
                acc[r][0][0] += w0[r]; acc[r][0][1] += w1[r]; acc[r][0][2] += w1[r + 1]; acc[r][0][3] += w0[r + 1];
                acc[r][1][0] += w1[r]; acc[r][1][1] += w2[r]; acc[r][1][2] += w2[r + 1]; acc[r][1][3] += w1[r + 1];
            }
        } else {
            const double* ck = scl + it.k * PER * PEC;
#pragma unroll
            for (int r = 0; r < PR + 1; ++r) {
                const pd2 c = *(const pd2*)(ck + r * PEC);
                acc[r][0][0] = fmadd(c.x, w0[r], acc[r][0][0]);
                acc[r][0][1] = fmadd(c.x, w1[r], acc[r][0][1]);
                acc[r][0][2] = fmadd(c.x, w1[r + 1], acc[r][0][2]);
                acc[r][0][3] = fmadd(c.x, w0[r + 1], acc[r][0][3]);
                acc[r][1][0] = fmadd(c.y, w1[r], acc[r][1][0]);
                acc[r][1][1] = fmadd(c.y, w2[r], acc[r][1][1]);
                acc[r][1][2] = fmadd(c.y, w2[r + 1], acc[r][1][2]);
                acc[r][1][3] = fmadd(c.y, w1[r + 1], acc[r][1][3]);
            }
        }
    };
    auto emit = [&](int j) {
        double* out = Yo + (int64_t)j * nodes;
        double kp[2][4];
#pragma unroll
        for (int r = 0; r < PR + 1; ++r) {
            double ka[4], kb[4];
            kref(acc[r][0][0], acc[r][0][1], acc[r][0][2], acc[r][0][3], ka[0], ka[1], ka[2], ka[3]);
            kref(acc[r][1][0], acc[r][1][1], acc[r][1][2], acc[r][1][3], kb[0], kb[1], kb[2], kb[3]);
            if (r > 0) {
                // node (x0, Y): elements (x0-1 | x0) x (Y-1 | Y); node (x0+1, Y): the pair's two elements
                const double left = dpp_from_left(kb[1] + kp[1][2]);
                const double n0 = (ka[0] + kp[0][3]) + left;
                const double n1 = (ka[1] + kp[0][2]) + (kb[0] + kp[1][3]);
                const int Yr = y0 - 1 + r;
                const bool yin = Yr >= 1 && Yr <= n - 1;
                if (Yr <= n) {
                    const int64_t qo = (int64_t)Yr * (n + 1) + x0;
                    const bool x0out = (gl >= 1 || x0 == 0) && x0 <= n;
                    const bool x1out = gl <= 30 && x0 + 1 <= n;
                    if (x0out) out[qo] = (yin && x0 >= 1 && x0 <= n - 1) ? n0 : 0.0;
                    if (x1out) out[qo + 1] = (yin && x0 + 1 <= n - 1) ? n1 : 0.0;
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                kp[0][c] = ka[c];
                kp[1][c] = kb[c];
            }
        }
#pragma unroll
        for (int r = 0; r < PR + 1; ++r)
#pragma unroll
            for (int e = 0; e < 2; ++e) acc[r][e][0] = acc[r][e][1] = acc[r][e][2] = acc[r][e][3] = 0.0;
    };
    // two input buffers: the loads of the next item are issued (unconditionally:
    // a branch around them would make the join wait for every load) before the
    // current item is accumulated
    pd2 A[PR + 2], B[PR + 2];
    todo = present(jc);
    PairItem cur;
    cur.col = jc; cur.g = c0; cur.k = -1; cur.j = jc; cur.last = todo == 0; cur.valid = true;
    load(A, cur.col);
#pragma unroll 1
    while (true) {
        PairItem nx = next_item();
        load(B, nx.valid ? nx.col : cur.col);
        __builtin_amdgcn_sched_barrier(0);
        accumulate(A, cur);
        if (cur.last) emit(cur.j);
        __builtin_amdgcn_sched_barrier(0);
        if (!nx.valid) break;
        cur = nx;
        nx = next_item();
        load(A, nx.valid ? nx.col : cur.col);
        __builtin_amdgcn_sched_barrier(0);
        accumulate(B, cur);
        if (cur.last) emit(cur.j);
        __builtin_amdgcn_sched_barrier(0);
        if (!nx.valid) break;
        cur = nx;
    }
}

SweepGeom make_geom(int n, int ncols, int64_t slices, int rows) {
    SweepGeom g;
    g.tiles_x = (n + 1 + GOUT - 1) / GOUT;
    g.tiles_y = (n + 1 + 2 * rows - 1) / (2 * rows);
    g.nchunks = (ncols + 3) / 4;
    const int64_t nb = slices * g.tiles_x * g.tiles_y * g.nchunks;
    if (nb > (int64_t)1 << 30) throw Error(SG_ERR_INVALID, "sweep launch grid too large");
    g.nb = (int)nb;
    return g;
}

}  // namespace

#define SG_ROWS_DISPATCH(rows, LAUNCH)                                                     \
    do {                                                                                   \
        switch (rows) {                                                                    \
            case 2: { constexpr int R = 2; LAUNCH; } break;                                \
            case 8: { constexpr int R = 8; LAUNCH; } break;                                \
            default: { constexpr int R = 4; LAUNCH; } break;                               \
        }                                                                                  \
    } while (0)

// Returns false when the sweep kernels do not cover the shape (M > 8).
template <typename T>
bool launch_sgx_apply(const Shape& s, const OpDev& op, const T* x, T* y, int nvec, uint32_t mask, hipStream_t st) {
    if (s.M > KMAX || s.field != SG_FIELD_AFFINE) return false;
    if constexpr (sizeof(T) == 8) {
        // FP64 storage: the paired-node kernel (strip height fixed)
        int tiles_x = 0;
        while (PGX * tiles_x + 1 <= s.n - 1) ++tiles_x;        // tile tx outputs node columns 62 tx + 1 .. 62 tx + 62
        const int tiles_y = (s.n + 1 + 2 * PR - 1) / (2 * PR);
        const int nchunks = (s.nxi + 4 * PNC - 1) / (4 * PNC);
        const int64_t nb = (int64_t)nvec * s.nt * tiles_x * tiles_y * nchunks;
        if (nb > (int64_t)1 << 30) throw Error(SG_ERR_INVALID, "SG apply launch grid too large");
        const int grid = (int)((nb + 7) / 8 * 8);
        hipLaunchKernelGGL(k_sgx_pair, dim3(grid), dim3(256), 0, st, s.n, s.M, s.nxi, s.nt, s.nodes, op, mask,
                           (const double*)x, (double*)y, tiles_x, tiles_y, nchunks, (int)nb);
        SG_HIP(hipGetLastError());
        return true;
    }
    ColMap z{};
    const int rows = s.sweep_rows[sizeof(T) == 4][SWEEP_APPLY];
    const SweepGeom g = make_geom(s.n, s.nxi, (int64_t)nvec * s.nt, rows);
    const int grid = (g.nb + 7) / 8 * 8;
    SG_ROWS_DISPATCH(rows, hipLaunchKernelGGL((k_sgx<T, 0, R, false>), dim3(grid), dim3(256), 0, st, s.n, s.M, s.nxi,
                                              s.nt, s.nodes, op, g, x, y, 0, 0, mask, 1, 1, (const T*)nullptr, z, z,
                                              z));
    SG_HIP(hipGetLastError());
    return true;
}

template <typename T>
bool launch_sgx_kkt(const Shape& s, const OpDev& op, const T* x, T* y, int nvec, hipStream_t st) {
    if (s.M > KMAX || s.field != SG_FIELD_AFFINE) return false;
    const int rows = s.sweep_rows[sizeof(T) == 4][SWEEP_KKT];
    const SweepGeom g = make_geom(s.n, s.nxi, (int64_t)nvec * s.nt, rows);
    const int grid = (g.nb + 7) / 8 * 8;
    if (s.time)
        SG_ROWS_DISPATCH(rows, hipLaunchKernelGGL((k_sgx_kkt<T, true, R>), dim3(grid), dim3(256), 0, st, s.n, s.M,
                                                  s.nxi, s.nt, s.nodes, op, g, x, y));
    else
        SG_ROWS_DISPATCH(rows, hipLaunchKernelGGL((k_sgx_kkt<T, false, R>), dim3(grid), dim3(256), 0, st, s.n, s.M,
                                                  s.nxi, s.nt, s.nodes, op, g, x, y));
    SG_HIP(hipGetLastError());
    return true;
}

template <typename T>
bool launch_sgx_hgs_rhs(const Shape& s, const OpDev& op, int d, uint32_t mask, int use_lower, int use_upper,
                        const T* base, ColMap bmap, const T* V, ColMap vmap, T* out, ColMap omap, int nmembers,
                        hipStream_t st) {
    if (s.M > KMAX || s.field != SG_FIELD_AFFINE) return false;
    const int L = s.off[d + 1] - s.off[d];
    const int rows = s.sweep_rows[sizeof(T) == 4][SWEEP_HGS];
    const SweepGeom g = make_geom(s.n, L, (int64_t)nmembers * s.nt, rows);
    const int grid = (g.nb + 7) / 8 * 8;
    // Alg. 1 sweeps one neighbour level at a time (forward: the lower level,
    // backward: the upper level), so every term has a single input column
    if (use_lower && use_upper) throw Error(SG_ERR_INVALID, "hGS right-hand side: one neighbour level at a time");
    SG_ROWS_DISPATCH(rows, hipLaunchKernelGGL((k_sgx<T, 1, R, false>), dim3(grid), dim3(256), 0, st, s.n, s.M, s.nxi,
                                              s.nt, s.nodes, op, g, V, out, s.off[d], L, mask, use_lower, use_upper,
                                              base, bmap, vmap, omap));
    SG_HIP(hipGetLastError());
    return true;
}

template bool launch_sgx_apply<double>(const Shape&, const OpDev&, const double*, double*, int, uint32_t, hipStream_t);
template bool launch_sgx_apply<float>(const Shape&, const OpDev&, const float*, float*, int, uint32_t, hipStream_t);
template bool launch_sgx_kkt<double>(const Shape&, const OpDev&, const double*, double*, int, hipStream_t);
template bool launch_sgx_kkt<float>(const Shape&, const OpDev&, const float*, float*, int, hipStream_t);
template bool launch_sgx_hgs_rhs<double>(const Shape&, const OpDev&, int, uint32_t, int, int, const double*, ColMap,
                                         const double*, ColMap, double*, ColMap, int, hipStream_t);
template bool launch_sgx_hgs_rhs<float>(const Shape&, const OpDev&, int, uint32_t, int, int, const float*, ColMap,
                                        const float*, ColMap, float*, ColMap, int, hipStream_t);

}  // namespace sg
