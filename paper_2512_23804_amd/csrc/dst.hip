// Exact solves with the mean block a K + b M and with the mass matrix M by the
// two-dimensional discrete sine transform, on FP64 MFMA.
//
// On the uniform n x n Q1 grid with homogeneous Dirichlet boundary the 1D
// stiffness K1 = n tridiag(-1, 2, -1) and mass M1 = (1/(6n)) tridiag(1, 4, 1)
// share the sine eigenvectors s_p(i) = sin(pi p i / n), p, i = 1..n-1, with
// eigenvalues k_p = 4 n sin^2(pi p / (2n)) and m_p = (2 + cos(pi p / n)) / (3n).
// The 2D operators K = K1 (x) M1 + M1 (x) K1 and M = M1 (x) M1 therefore have
// eigenvalues a (k_p m_q + m_p k_q) + b m_p m_q on the products of sines, and
// with S = [s_p(i)] (S^2 = (n/2) I):
//   (a K + b M)^{-1} B = (2/n)^2 S [ (S B S) ./ lambda ] S.
// This holds because the mean coefficient kappa_0 is constant (the mean block
// of eq. mathcalZ / eq. A_hat is a K_unit + b M) and M is the unweighted mass
// matrix of the Q1 space.
//
// Each of the four products is one pass of out_c = (S in_c)^T over a batch of
// columns (two passes give S B S); a block computes a 64 x 64 tile of S in_c
// with sixteen FP64 16x16x4 MFMA tiles per k-chunk of 16 (S generated from a
// table of sin(pi m / n), m < 2n; the input chunk staged in LDS), and writes
// the transposed tile through LDS so that the stores are row-contiguous.  The
// second pass divides by the eigenvalues (and applies the column scale of the
// mass blocks); intermediate products are FP64 whatever the storage type.
#include "common.hpp"

namespace sg {

namespace {

constexpr int DT = 64;    // output tile side
constexpr int DK = 16;    // k-chunk

struct DstEpi {
    const MemberDev* mem;   // per-member scalars (mean block a1, b1; mass scalings)
    const double* eig;      // [2][n+1]: k_p, m_p
    int mode;               // 0: none; 1: divide by a1 (k m + m k) + b1 m m (member c / cpm); 2: mass (m m), column scale
    int shared;             // mode 2: every vector uses member 0
    int cpm;                // columns per member constants (mode 1)
    int nt, nxi, time;      // mode 2: column l = c % (2 nt nxi) -> block, t, j
    double f;               // (2/n)^2
};

// out_c[j][i] = sum_k S[i][k] in_c[k][j] over interior indices i, j, k = 1..n-1
// (ring of out untouched); EPI applies the eigenvalue division on (i, j).
template <typename TI, typename TO, bool EPI>
__global__ __launch_bounds__(256) void k_dst_pass(int n, const TI* __restrict__ in, ColMap imap, TO* __restrict__ out,
                                                  ColMap omap, const double* __restrict__ sintab, DstEpi ep,
                                                  int tiles, const int* __restrict__ act, int cpv) {
    typedef double v4d __attribute__((ext_vector_type(4)));
    const int c = blockIdx.y;
    if (act && !act[c / cpv]) return;                 // uniform per block, before any barrier
    const int ti = blockIdx.x % tiles, tj = blockIdx.x / tiles;
    const int i0 = 1 + ti * DT, j0 = 1 + tj * DT;
    const int N1 = n + 1, n2 = 2 * n;
    __shared__ double sS[DT][DK + 1];                 // S[i0 + r][k0 + kk]
    __shared__ double sI[DK][DT + 1];                 // in[k0 + kk][j0 + cc]
    __shared__ double sO[DT][DT + 1];                 // transposed output tile
    const TI* src = in + imap.off(c);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int l16 = lane & 15, lq = lane >> 4;
    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 1; k0 <= n - 1; k0 += DK) {
        double vs[4], vi[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = tid + 256 * e;
            const int r = q / DK, kk = q % DK;        // S tile 64 x 16
            const int i = i0 + r, k = k0 + kk;
            vs[e] = (i <= n - 1 && k <= n - 1) ? sintab[(i * k) % n2] : 0.0;
            const int kr = q / DT, cc = q % DT;       // input tile 16 x 64
            const int kk2 = k0 + kr, j = j0 + cc;
            vi[e] = (kk2 <= n - 1 && j <= n - 1) ? (double)src[(int64_t)kk2 * N1 + j] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = tid + 256 * e;
            sS[q / DK][q % DK] = vs[e];
            sI[q / DT][q % DT] = vi[e];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < DK; ks += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = sS[wr + a * 16 + l16][ks + lq];     // A[row][k]
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = sI[ks + lq][wc + b * 16 + l16];     // B[k][col]
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // acc[a][b][q] holds D[row = wr + 16a + lane/16 + 4q][col = wc + 16b + lane%16] (FP64 16x16x4
    // output layout), D = S in over the tile; stage D^T in LDS
    double cf = 1.0;
    int mem = 0;
    if (EPI) {
        if (ep.mode == 1) {
            mem = c / ep.cpm;
        } else {
            const int per = 2 * ep.nt * ep.nxi;
            const int vec = c / per, l = c % per;
            const int var = l / (ep.nt * ep.nxi), t = (l / ep.nxi) % ep.nt, j = l % ep.nxi;
            mem = ep.shared ? 0 : vec;
            const MemberDev md = ep.mem[mem];
            const double Dt = (ep.time && (t == 0 || t == ep.nt - 1)) ? 0.5 : 1.0;
            const double sc = var == 0 ? (j == 0 ? 1.0 : md.hg) : md.beta;
            cf = 1.0 / (sc * md.tau * Dt);
        }
    }
    const double a1 = EPI && ep.mode == 1 ? ep.mem[mem].a1 : 0.0;
    const double b1 = EPI && ep.mode == 1 ? ep.mem[mem].b1 : 1.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = wr + 16 * a + lq + 4 * q, col = wc + 16 * b + l16;
                double v = acc[a][b][q];
                if (EPI) {
                    const int p = min(i0 + row, n - 1), r = min(j0 + col, n - 1);
                    const double kp = ep.eig[p], mp = ep.eig[N1 + p], kr = ep.eig[r], mr = ep.eig[N1 + r];
                    const double lam = a1 * (kp * mr + mp * kr) + b1 * (mp * mr);
                    v = v * (ep.f * cf / lam);
                }
                sO[col][row] = v;
            }
    __syncthreads();
    TO* dst = out + omap.off(c);
    for (int q = tid; q < DT * DT; q += 256) {
        const int jj = q / DT, ii = q % DT;
        const int j = j0 + jj, i = i0 + ii;
        if (j <= n - 1 && i <= n - 1) dst[(int64_t)j * N1 + i] = (TO)sO[jj][ii];
    }
}

// the ring (i or j = 0 or n) of each output column set to zero
template <typename T>
__global__ void k_dst_ring(int n, T* __restrict__ out, ColMap omap, const int* __restrict__ act, int cpv) {
    const int c = blockIdx.y;
    if (act && !act[c / cpv]) return;
    const int N1 = n + 1;
    T* dst = out + omap.off(c);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < 4 * N1; q += gridDim.x * blockDim.x) {
        const int side = q / N1, e = q % N1;
        const int64_t p = side == 0 ? e : side == 1 ? (int64_t)n * N1 + e : side == 2 ? (int64_t)e * N1
                                                                                     : (int64_t)e * N1 + n;
        dst[p] = T(0);
    }
}

template <typename TI, typename TO, bool EPI>
void dst_pass(int n, const TI* in, ColMap imap, TO* out, ColMap omap, const double* sintab, const DstEpi& ep,
              int ncols, const int* act, int cpv, hipStream_t st) {
    const int tiles = (n - 1 + DT - 1) / DT;
    hipLaunchKernelGGL((k_dst_pass<TI, TO, EPI>), dim3(tiles * tiles, ncols), dim3(256), 0, st, n, in, imap, out,
                       omap, sintab, ep, tiles, act, cpv);
}

}  // namespace

template <typename T>
void launch_dst_solve(int n, int mode, const MemberDev* mem, int shared, const double* sintab, const double* eig,
                      const T* b,
                      ColMap bmap, T* x, ColMap xmap, int ncols, int cpm, int nt, int nxi, int time, double* s1,
                      double* s2, const int* act, int cpv, hipStream_t st) {
    if (ncols < 1) return;
    if (ncols > 65535) throw Error(SG_ERR_INVALID, "sine-transform solve: too many columns in one launch");
    const int64_t nodes = (int64_t)(n + 1) * (n + 1);
    const ColMap cm = contiguous_cols(ncols, nodes);
    DstEpi none{};
    DstEpi ep{mem, eig, mode, shared, cpm, nt, nxi, time, 4.0 / ((double)n * n)};
    dst_pass<T, double, false>(n, b, bmap, s1, cm, sintab, none, ncols, act, cpv, st);        // (S B)^T
    dst_pass<double, double, true>(n, s1, cm, s2, cm, sintab, ep, ncols, act, cpv, st);      // S B S ./ lambda
    dst_pass<double, double, false>(n, s2, cm, s1, cm, sintab, none, ncols, act, cpv, st);
    dst_pass<double, T, false>(n, s1, cm, x, xmap, sintab, none, ncols, act, cpv, st);
    hipLaunchKernelGGL((k_dst_ring<T>), dim3(4, ncols), dim3(256), 0, st, n, x, xmap, act, cpv);
    SG_HIP(hipGetLastError());
}

template void launch_dst_solve<double>(int, int, const MemberDev*, int, const double*, const double*, const double*, ColMap,
                                       double*, ColMap, int, int, int, int, int, double*, double*, const int*, int,
                                       hipStream_t);
template void launch_dst_solve<float>(int, int, const MemberDev*, int, const double*, const double*, const float*, ColMap,
                                      float*, ColMap, int, int, int, int, int, double*, double*, const int*, int,
                                      hipStream_t);

}  // namespace sg
