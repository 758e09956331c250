// Operator tables built on the device: banded LU factors of every radial
// operator (Section 2: the implicit viscous terms and the pressure-Poisson
// equation are solved by banded LU per Fourier mode), the homogeneous
// solutions and inverse influence matrices of the influence-matrix
// correction, and the flux Green's function.  They are built when a context
// is created and again whenever the step size changes (the Helmholtz
// operators H = 1/dt - (c/Re) L depend on dt).
#include <cmath>

#include "opf_internal.h"

namespace opf {
namespace {

constexpr int BW = 13;  // band entries per row: offsets -8..+4 from the diagonal

__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Twisted elimination of the band held in T (N = NB rows, offsets -8..+4)
// and the twisted substitution image (layout and scaling as described at
// solve_twisted): columns 0..h-1 top-down (lane t updates row j+1+t/4,
// column j+1+t%4), columns NB-1..h+4 bottom-up (lane t updates row
// j-1-t/8, column j-8+t%8), both without pivoting; the multipliers replace
// the eliminated entries.  The middle block is inverted by Gauss-Jordan with
// row pivoting.  Called by all 64 lanes.
__device__ void twisted_image(const FactorArgs& a, double* T, double* G, double* Dv, double amax, int& bad) {
    const int N = a.N, NB = a.NB, h = tw_h(NB), n = threadIdx.x;
    for (int j = 0; j < h; ++j) {
        const double piv = T[j * BW + 8];
        if (!(fabs(piv) > 1e-14 * amax)) bad = bad ? bad : 2;
        const int i = j + 1 + (n & 31) / 4, col = j + 1 + (n & 3);
        if (n < 32 && i < N) {
            const double l = T[i * BW + (j - i + 8)] / piv;
            if (col < N && col - i >= -8) T[i * BW + (col - i + 8)] -= l * T[j * BW + (col - j + 8)];
            if ((n & 3) == 0) T[i * BW + (j - i + 8)] = l;
        }
        __syncthreads();
    }
    for (int j = N - 1; j >= h + 4; --j) {
        const double piv = T[j * BW + 8];
        if (!(fabs(piv) > 1e-14 * amax)) bad = bad ? bad : 2;
        const int i = j - 1 - (n & 31) / 8, col = j - 8 + (n & 7);
        if (n < 32 && i >= 0) {
            const double u = T[i * BW + (j - i + 8)] / piv;
            if (col >= 0) T[i * BW + (col - i + 8)] -= u * T[j * BW + (col - j + 8)];
            if ((n & 7) == 0) T[i * BW + (j - i + 8)] = u;
        }
        __syncthreads();
    }
    // element growth of the eliminated rows (the multipliers left out: the
    // bottom-up ones against the identity wall row are the wall stencil's
    // entries themselves, large by construction and exact)
    double g = 0.0;
    if (n < N) {
        const int lo = n < h ? n : (n < h + 4 ? h : max(n - 8, 0)), hi = n < h ? n + 4 : (n < h + 4 ? h + 3 : n);
        for (int c = lo; c <= hi && c < N; ++c) g = fmax(g, fabs(T[n * BW + (c - n + 8)]));
    }
    if (wave_max(g) > 1e3 * amax) bad = bad ? bad : 3;
    auto sv = [&](int i) { return i >= h && i < h + 4 ? 1.0 : 1.0 / T[i * BW + 8]; };
    if (n == 0) {
        double m[4][8];
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                m[r][c] = T[(h + r) * BW + (c - r + 8)];
                m[r][4 + c] = r == c ? 1.0 : 0.0;
            }
        for (int c = 0; c < 4; ++c) {
            int pr = c;
            for (int r = c + 1; r < 4; ++r)
                if (fabs(m[r][c]) > fabs(m[pr][c])) pr = r;
            if (!(fabs(m[pr][c]) > 1e-14 * amax)) bad = bad ? bad : 2;
            if (pr != c)
                for (int e = 0; e < 8; ++e) {
                    const double x = m[c][e];
                    m[c][e] = m[pr][e];
                    m[pr][e] = x;
                }
            const double inv = 1.0 / m[c][c];
            for (int e = 0; e < 8; ++e) m[c][e] *= inv;
            for (int r = 0; r < 4; ++r)
                if (r != c) {
                    const double f = m[r][c];
                    for (int e = 0; e < 8; ++e) m[r][e] -= f * m[c][e];
                }
        }
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) G[tw_mi(NB) + 4 * r + c] = m[r][4 + c];
    }
    if (n < h) {
        const int t = n, j = NB - 1 - t;
        for (int d = 0; d < 4; ++d) {
            const int i = t + 1 + d, ib = j - 1 - d;
            G[4 * t + d] = sv(i) * T[i * BW + (t - i + 8)] * T[t * BW + 8];
            G[tw_p1b(NB) + 4 * t + d] = sv(ib) * T[ib * BW + (j - ib + 8)] * T[j * BW + 8];
        }
    }
    if (n < 4) G[tw_z4(NB) + n] = 0.0;
    if (n < h + 4) {
        const int t = n, ja = h + 3 - t, jb = h + t;
        for (int d = 0; d < 4; ++d) {
            const int i = ja - 1 - d;
            G[tw_p3a(NB) + 4 * t + d] = i >= 0 && i < h ? T[i * BW + (ja - i + 8)] * sv(i) : 0.0;
        }
        double* g = G + tw_p3b_rec(NB, t);
        for (int d = 0; d < (tw_wide(NB, t) ? 8 : 4); ++d) {
            const int i = jb + 1 + d;
            g[d] = i >= h + 4 && i < NB ? T[i * BW + (jb - i + 8)] * sv(i) : 0.0;
        }
    }
    if (n < NB) Dv[n] = sv(n);
}

// One system per 64-thread workgroup.  System q < MU K is H_{mu,|k|} with
// mu = q / K, |k| = q % K; q >= MU K is the pressure operator L_{m,|k|},
// m = mp (q - MU K) / K, with P(1) = 0 (the unused (0,0) record gets
// 1/U = 1).  The band (rows in LDS) is eliminated without pivoting, one
// column per pass (8 rows x 4 columns of updates in parallel), then written
// as column records: main record i holds L[i+1..i+4][i], U[i-1..i-4][i] and
// 1/U_ii, tail record i holds L[i+5..i+8][i].  flags[q]: 0 ok, 1 entry outside the band, 2 pivot below
// 1e-14 max|A|, 3 element growth (|U| > 1e3 max|A| or |L| > 1e3).
__global__ __launch_bounds__(64) void k_factor(FactorArgs a, int first) {
    __shared__ double B[NMAX * BW];
    __shared__ double T[NMAX * BW];  // the band again, for the twisted elimination
    const int q = first + blockIdx.x;
    const int N = a.N, n = threadIdx.x;
    const bool helm = q < a.MU * a.K;
    const int mu = helm ? q / a.K : a.mp * ((q - a.MU * a.K) / a.K);
    const int ka = helm ? q % a.K : (q - a.MU * a.K) % a.K;
    double* F = a.fac + (size_t)q * N * FACW;
    // substitution image of this operator: [|k|][mu] (Helmholtz), [|k|][m] (pressure)
    const int FW = solve_image_doubles(a.NB, a.NW), FWD = solve_image_fwd(a.NB, a.NW);
    const size_t iq = helm ? (size_t)ka * a.MU + mu : (size_t)a.MU * a.K + (size_t)ka * a.M + (q - a.MU * a.K) / a.K;
    double* G = a.img + iq * FW;
    double* Dv = a.dinv + iq * a.NB;
    if (!helm && mu == 0 && ka == 0) {
        if (n < N) {
            for (int d = 0; d < FMAIN; ++d) F[(size_t)n * FMAIN + d] = d == 8 ? 1.0 : 0.0;
            for (int d = 0; d < FTAIL; ++d) F[(size_t)N * FMAIN + (size_t)n * FTAIL + d] = 0.0;
        }
        for (int e = n; e < FW; e += 64) G[e] = 0.0;
        if (n < a.NB) Dv[n] = 0.0;
        if (n == 0) a.flags[q] = 0;
        return;
    }
    const double kap = a.alpha * ka;
    const int par = mu & 1;
    int bad = 0;
    double amax = 0.0;
    if (n < N) {
        for (int d = 0; d < BW; ++d) B[n * BW + d] = 0.0;
        if (n == N - 1) {
            B[n * BW + 8] = 1.0;  // wall row: the boundary value
            amax = 1.0;
        } else {
            const int s = a.s0[n];
            const double ri = a.rinv[n];
            for (int j = 0; j < W9; ++j) {
                const int col = s + j;
                double v = a.d2[(par * N + n) * W9 + j] + ri * a.d1[(par * N + n) * W9 + j];
                if (col == n) v -= double(mu) * mu * ri * ri + kap * kap;
                if (helm) {
                    v = -a.cr * v;
                    if (col == n) v += a.inv_dt;
                }
                const int off = col - n;
                if (off < -8 || off > 4) {
                    if (v != 0.0) bad = 1;
                } else {
                    B[n * BW + off + 8] = v;
                }
                amax = fmax(amax, fabs(v));
            }
        }
    }
    amax = wave_max(amax);
    __syncthreads();
    const bool tw = solve_twisted(a.NB, a.NW);
    if (tw) {
        for (int e = n; e < N * BW; e += 64) T[e] = B[e];
        if (N != a.NB) bad = 1;  // the twisted images assume N = NB
    }
    __syncthreads();
    // elimination: lane t updates row j+1+t/4, column j+1+t%4
    const int ti = 1 + (n & 31) / 4, tc = 1 + (n & 3);
    for (int j = 0; j < N; ++j) {
        const double piv = B[j * BW + 8];
        if (!(fabs(piv) > 1e-14 * amax)) bad = bad ? bad : 2;
        const int i = j + ti, col = j + tc;
        if (n < 32 && i < N) {
            const double l = B[i * BW + (j - i + 8)] / piv;
            if (col < N && col - i >= -8) B[i * BW + (col - i + 8)] -= l * B[j * BW + (col - j + 8)];
            if (tc == 1) B[i * BW + (j - i + 8)] = l;
        }
        __syncthreads();
    }
    double umax = 0.0, lmax = 0.0;
    if (n < N)
        for (int d = 0; d < BW; ++d) {
            const double v = fabs(B[n * BW + d]);
            if (d >= 8) umax = fmax(umax, v);
            else lmax = fmax(lmax, v);
        }
    umax = wave_max(umax);
    lmax = wave_max(lmax);
    if (n < N) {
        double* f = F + (size_t)n * FMAIN;
        double* tl = F + (size_t)N * FMAIN + (size_t)n * FTAIL;
        for (int d = 0; d < 8; ++d) {
            const double l = n + 1 + d < N ? B[(n + 1 + d) * BW + (7 - d)] : 0.0;
            if (d < 4) f[d] = l;
            else tl[d - 4] = l;
        }
        for (int d = 0; d < 4; ++d) f[4 + d] = n - 1 - d >= 0 ? B[(n - 1 - d) * BW + (9 + d)] : 0.0;
        f[8] = 1.0 / B[n * BW + 8];
        f[9] = 0.0;
    }
    // image: Lh[n+d][n] = L[n+d][n] U_nn / U_{n+d,n+d}, W[n-d][n] = U[n-d][n] / U_{n-d,n-d}
    if (tw) {
        twisted_image(a, T, G, Dv, amax, bad);
    } else if (n < a.NB) {
        const int nd = n < a.NW ? 4 : 8;
        double* g = G + (n < a.NW ? 4 * n : 4 * a.NW + 8 * (n - a.NW));
        for (int d = 1; d <= nd; ++d)
            g[d - 1] = n < N && n + d < N ? B[(n + d) * BW + (8 - d)] * B[n * BW + 8] / B[(n + d) * BW + 8] : 0.0;
        if (n >= 1) {
            double* gb = G + FWD + 4 * (n - 1);
            for (int d = 1; d <= 4; ++d)
                gb[d - 1] = n < N && n - d >= 0 ? B[(n - d) * BW + (8 + d)] / B[(n - d) * BW + 8] : 0.0;
        }
        Dv[n] = n < N ? 1.0 / B[n * BW + 8] : 0.0;
    }
    // the band check is per row: any lane's flag marks the system
    for (int o = 32; o > 0; o >>= 1) bad = max(bad, __shfl_xor(bad, o));
    if (bad == 0 && (umax > 1e3 * amax || lmax > 1e3)) bad = 3;
    if (n == 0) a.flags[q] = bad;
}

// Forward and backward substitution with column records, on a vector held
// in LDS column `lane` of v[n * 64 + lane].
__device__ void rec_solve(const double* __restrict__ F, int N, double* v, int lane) {
    for (int i = 0; i < N; ++i) {
        const double* f = F + (size_t)i * FMAIN;
        const double* tl = F + (size_t)N * FMAIN + (size_t)i * FTAIL;
        const double x = v[i * 64 + lane];
        for (int d = 0; d < 8; ++d)
            if (i + 1 + d < N) v[(i + 1 + d) * 64 + lane] -= (d < 4 ? f[d] : tl[d - 4]) * x;
    }
    for (int i = N - 1; i >= 0; --i) {
        const double* f = F + (size_t)i * FMAIN;
        const double x = v[i * 64 + lane] * f[8];
        v[i * 64 + lane] = x;
        for (int d = 0; d < 4; ++d)
            if (i - 1 - d >= 0) v[(i - 1 - d) * 64 + lane] -= f[4 + d] * x;
    }
}

__device__ inline const double* hfac(const FactorArgs& a, int mu, int ka) {
    return a.fac + ((size_t)abs(mu) * a.K + ka) * a.N * FACW;
}

// P1 = L_{m,|k|}^{-1} e_{N-1} (unit wall pressure) into slot 6 of the
// influence data; the (0,0) pair gets zeros in every slot.  One thread per
// (m, |k|) pair.
__global__ __launch_bounds__(64) void k_hom_pressure(FactorArgs a) {
    __shared__ double v[NMAX * 64];
    const int lane = threadIdx.x, pr = blockIdx.x * 64 + lane;
    const int N = a.N;
    if (pr >= a.M * a.K) return;
    const int mi = pr / a.K, ka = pr % a.K;
    double* h = a.hom + (size_t)pr * NHOM * N;
    if (mi == 0 && ka == 0) {
        for (int s = 0; s < NHOM * N; ++s) h[s] = 0.0;
        return;
    }
    for (int i = 0; i < N; ++i) v[i * 64 + lane] = i == N - 1 ? 1.0 : 0.0;
    rec_solve(a.fac + ((size_t)a.MU * a.K + pr) * N * FACW, N, v, lane);
    for (int i = 0; i < N; ++i) h[6 * N + i] = v[i * 64 + lane];
}

// The six Helmholtz solves of the homogeneous solutions of pair (m, |k|):
// slot 0 h1+ = H_{m+1}^{-1}(-(P1' - m P1/r)), slot 1 h1- = H_{m-1}^{-1}(-(P1'
// + m P1/r)), slot 2 q = H_m^{-1} P1 (wall values 0), and slots 3..5 the unit
// wall values through H_{m+1}, H_{m-1}, H_m.  One thread per (pair, slot).
__global__ __launch_bounds__(64) void k_hom_helmholtz(FactorArgs a) {
    __shared__ double v[NMAX * 64];
    const int lane = threadIdx.x, id = blockIdx.x * 64 + lane;
    const int N = a.N;
    if (id >= a.M * a.K * 6) return;
    const int pr = id / 6, slot = id % 6;
    const int mi = pr / a.K, ka = pr % a.K;
    if (mi == 0 && ka == 0) return;
    const int m = a.mp * mi;
    double* h = a.hom + (size_t)pr * NHOM * N;
    const double* P1 = h + 6 * N;
    for (int i = 0; i < N; ++i) {
        double r = 0.0;
        if (i == N - 1) {
            r = slot >= 3 ? 1.0 : 0.0;
        } else if (slot < 2) {
            double dP = 0.0;
            for (int j = 0; j < W9; ++j) dP += a.d1[((m & 1) * N + i) * W9 + j] * P1[a.s0[i] + j];
            const double t = m * P1[i] * a.rinv[i];
            r = slot == 0 ? -(dP - t) : -(dP + t);
        } else if (slot == 2) {
            r = P1[i];
        }
        v[i * 64 + lane] = r;
    }
    const int mu = (slot == 0 || slot == 3) ? m + 1 : (slot == 1 || slot == 4) ? m - 1 : m;
    rec_solve(hfac(a, mu, ka), N, v, lane);
    for (int i = 0; i < N; ++i) h[slot * N + i] = v[i * 64 + lane];
}

struct c2 {
    double x, y;
};
__device__ inline c2 cmul(c2 p, c2 q) { return {p.x * q.x - p.y * q.y, p.x * q.y + p.y * q.x}; }
__device__ inline c2 csub(c2 p, c2 q) { return {p.x - q.x, p.y - q.y}; }
__device__ inline double cabs2(c2 p) { return sqrt(p.x * p.x + p.y * p.y); }
__device__ inline c2 cdiv(c2 p, c2 q) {
    const double d = q.x * q.x + q.y * q.y;
    return {(p.x * q.x + p.y * q.y) / d, (p.y * q.x - p.x * q.y) / d};
}

// Inverse influence matrix of mode (m, k): A_ij = g_i(h_j) with
// g(v) = (v+(1), v-(1), v_z(1), div v(1)) and h_1 = (h1+, h1-, -i kappa q),
// h_2..h_4 the unit wall solutions, inverted by Gauss-Jordan elimination
// with partial pivoting.  One thread per (m, signed k); (0,0) gets zeros,
// and a singular matrix sets flags[mode].
__global__ __launch_bounds__(64) void k_influence(FactorArgs a) {
    int* flags = a.flags + a.MU * a.K + a.M * a.K;
    const int id = blockIdx.x * 64 + threadIdx.x;
    const int N = a.N, K = a.K, nk = 2 * K - 1;
    if (id >= a.M * nk) return;
    const int mi = id / nk, k = id % nk - (K - 1), ka = abs(k);
    double* dst = a.ainv + (size_t)id * 32;
    flags[id] = 0;
    if (mi == 0 && ka == 0) {
        for (int s = 0; s < 32; ++s) dst[s] = 0.0;
        return;
    }
    const int m = a.mp * mi, e = N - 1, po = (m + 1) & 1;
    const double kap = a.alpha * k, re = a.rinv[e];
    const double* h = a.hom + ((size_t)mi * K + ka) * NHOM * N;
    auto d1row = [&](const double* v) {
        double acc = 0.0;
        for (int j = 0; j < W9; ++j) acc += a.d1[(po * N + e) * W9 + j] * v[a.s0[e] + j];
        return acc;
    };
    const double* h1p = h;
    const double* h1m = h + N;
    const double* q = h + 2 * N;
    const double* h2 = h + 3 * N;
    const double* h3 = h + 4 * N;
    const double* h4 = h + 5 * N;
    const double dp1 = 0.5 * (d1row(h1p) + (1 + m) * h1p[e] * re) + 0.5 * (d1row(h1m) + (1 - m) * h1m[e] * re);
    c2 A[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) A[i][j] = {j - 4 == i ? 1.0 : 0.0, 0.0};
    A[0][0] = {h1p[e], 0.0};
    A[1][0] = {h1m[e], 0.0};
    A[2][0] = {0.0, -kap * q[e]};               // -i kappa q
    A[3][0] = {dp1 + kap * kap * q[e], 0.0};    // div h1: + i kappa (-i kappa q)
    A[0][1] = {h2[e], 0.0};
    A[3][1] = {0.5 * (d1row(h2) + (1 + m) * h2[e] * re), 0.0};
    A[1][2] = {h3[e], 0.0};
    A[3][2] = {0.5 * (d1row(h3) + (1 - m) * h3[e] * re), 0.0};
    A[2][3] = {h4[e], 0.0};
    A[3][3] = {0.0, kap * h4[e]};               // i kappa h4
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int i = c + 1; i < 4; ++i)
            if (cabs2(A[i][c]) > cabs2(A[piv][c])) piv = i;
        if (cabs2(A[piv][c]) == 0.0) {
            flags[id] = 1;
            for (int s = 0; s < 32; ++s) dst[s] = 0.0;
            return;
        }
        for (int j = 0; j < 8; ++j) {
            const c2 t = A[c][j];
            A[c][j] = A[piv][j];
            A[piv][j] = t;
        }
        const c2 d = A[c][c];
        for (int j = 0; j < 8; ++j) A[c][j] = cdiv(A[c][j], d);
        for (int i = 0; i < 4; ++i)
            if (i != c) {
                const c2 f = A[i][c];
                for (int j = 0; j < 8; ++j) A[i][j] = csub(A[i][j], cmul(f, A[c][j]));
            }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            dst[2 * (4 * i + j)] = A[i][4 + j].x;
            dst[2 * (4 * i + j) + 1] = A[i][4 + j].y;
        }
}

// Flux Green's function H_{0,0} u_G = 1 inside, u_G(1) = 0, and
// qg = int_0^1 u_G r dr (one thread).
__global__ __launch_bounds__(64) void k_green(FactorArgs a, double* qg) {
    __shared__ double v[NMAX * 64];
    if (threadIdx.x != 0) return;
    const int N = a.N;
    for (int i = 0; i < N; ++i) v[i * 64] = i == N - 1 ? 0.0 : 1.0;
    rec_solve(hfac(a, 0, 0), N, v, 0);
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
        a.green[i] = v[i * 64];
        s += a.quad[i] * v[i * 64];
    }
    *qg = s;
}

}  // namespace

hipError_t launch_operator_tables(const FactorArgs& a, bool pressure, hipStream_t s) {
    const int nh = a.MU * a.K, np = a.M * a.K;
    hipLaunchKernelGGL(k_factor, dim3(pressure ? nh + np : nh), dim3(64), 0, s, a, 0);
    hipError_t he = hipGetLastError();
    if (he != hipSuccess) return he;
    if (pressure) {
        hipLaunchKernelGGL(k_hom_pressure, dim3((np + 63) / 64), dim3(64), 0, s, a);
        if ((he = hipGetLastError()) != hipSuccess) return he;
    }
    hipLaunchKernelGGL(k_hom_helmholtz, dim3((np * 6 + 63) / 64), dim3(64), 0, s, a);
    if ((he = hipGetLastError()) != hipSuccess) return he;
    const int modes = a.M * (2 * a.K - 1);
    hipLaunchKernelGGL(k_influence, dim3((modes + 63) / 64), dim3(64), 0, s, a);
    if ((he = hipGetLastError()) != hipSuccess) return he;
    hipLaunchKernelGGL(k_green, dim3(1), dim3(64), 0, s, a, a.qg);
    return hipGetLastError();
}

}  // namespace opf
