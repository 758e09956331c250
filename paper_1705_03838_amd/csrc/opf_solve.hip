// Radial solves of one substep on MI355X: right-hand side, pressure-Poisson
// equation, Helmholtz equations, influence-matrix boundary correction,
// fixed flux and vorticity, for every Fourier mode.
//
// Section 2 of the paper: a pressure-Poisson formulation with an influence-
// matrix enforcement of the boundary conditions (g = 0 when satisfied);
// Section 2.2: the implicit viscous terms are banded systems solved by LU
// decomposition for each Fourier mode.  With u+- = u_r +- i u_theta the
// vector Laplacian decouples (L_{m+-1} on u+-, L_m on u_z and P), so every
// system is a real banded matrix acting on complex data.
//
// One 4-wave workgroup handles |k| and GM consecutive m (GM = 4 for mp = 1),
// both signs of k: up to eight modes, which share their factors (they depend
// on |k|, and neighbouring m share Helmholtz operators).  Lanes are radial
// nodes for the stencil work, wave w holding modes 2w and 2w+1; for the
// substitutions each lane of wave 0 owns one real right-hand side (a real or
// imaginary part of one component of one mode) and walks the rows with the
// factor staged in LDS.  m = 0 solves k >= 0 only and writes the conjugate
// into -k (Hermitian symmetry of a real field); mode (0,0) has u_r = 0, no
// pressure and the fixed-flux correction.
#include "opf_internal.h"

namespace opf {

constexpr int LSTR = NMAX + 2;            // LDS line stride (complex): avoids bank aliasing

struct dcplx {
    double x, y;
};
__device__ __forceinline__ dcplx operator+(dcplx a, dcplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ dcplx operator-(dcplx a, dcplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ dcplx operator*(double s, dcplx a) { return {s * a.x, s * a.y}; }
__device__ __forceinline__ dcplx cm(dcplx a, dcplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ dcplx ix(dcplx a) { return {-a.y, a.x}; }  // i * a

// Row n of a 9-point stencil applied to a radial line in LDS.
__device__ __forceinline__ dcplx stencil(const double* w, const dcplx* line, int s0) {
    dcplx acc = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < W9; ++j) acc = acc + w[j] * line[s0 + j];
    return acc;
}

// Row weights of both axis parities held in registers (one lane = one row).
struct RowW {
    double e[W9], o[W9];
    __device__ __forceinline__ void load(const double* tab, int N, int n) {
#pragma unroll
        for (int j = 0; j < W9; ++j) {
            e[j] = tab[n * W9 + j];
            o[j] = tab[(N + n) * W9 + j];
        }
    }
    __device__ __forceinline__ dcplx apply(int par, const dcplx* line, int s0) const {
        dcplx acc = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < W9; ++j) acc = acc + (par ? o[j] : e[j]) * line[s0 + j];
        return acc;
    }
};

template <typename T>
__device__ __forceinline__ dcplx load_c(const void* base, size_t idx) {
    const T* p = reinterpret_cast<const T*>(base) + 2 * idx;
    return {double(p[0]), double(p[1])};
}
template <typename T>
__device__ __forceinline__ void store_c(void* base, size_t idx, dcplx v) {
    T* p = reinterpret_cast<T*>(base) + 2 * idx;
    p[0] = T(v.x);
    p[1] = T(v.y);
}

// Vorticity at row n from (+,-,z) lines (Section 2.2, rotational form):
//   w+ = (i m / r) u_z - i u_z' - kappa u+,   w- = (i m / r) u_z + i u_z' + kappa u-,
//   w_z = -(i/2)[u+' + (1+m) u+ / r] + (i/2)[u-' + (1-m) u- / r].
__device__ __forceinline__ void vort_row(const Tables& t, int N, int n, int m, double kap,
                                         const dcplx* up, const dcplx* um, const dcplx* uz,
                                         dcplx& wp, dcplx& wm, dcplx& wz) {
    const int pe = m & 1, po = (m + 1) & 1;
    const int s0 = t.s0[n];
    const double rinv = t.rinv[n];
    const dcplx duz = stencil(t.d1 + (pe * N + n) * W9, uz, s0);
    const dcplx dup = stencil(t.d1 + (po * N + n) * W9, up, s0);
    const dcplx dum = stencil(t.d1 + (po * N + n) * W9, um, s0);
    const dcplx imz = (double(m) * rinv) * ix(uz[n]);
    wp = imz - ix(duz) - kap * up[n];
    wm = imz + ix(duz) + kap * um[n];
    const dcplx ap = dup + (double(1 + m) * rinv) * up[n];
    const dcplx am = dum + (double(1 - m) * rinv) * um[n];
    wz = 0.5 * ix(am - ap);
}

// Substitution for one real right-hand side living in LDS (`col`, element i
// at col[2 i]) with a factor in LDS whose row record i holds column i of L
// below the diagonal (8 values), column i of U above it (4 values) and
// 1/U_ii.  Right-looking: once y_i is known it updates the next 8 entries,
// kept in registers, so only one FMA per row lies on the dependency chain;
// factor records and right-hand-side entries are fetched PF rows ahead.
// Rows N..NB-1 of the factor and of `col` are zero (the padded tail stays
// zero; no branches).  Columns j < NW have no nonzero L entry more than four
// rows below the diagonal (SolveArgs::narrow >= NW): their rows read and
// apply only the first four, with the same result.  With all but the last
// nine rows narrow, records are fetched 5 rows ahead instead of 3; with
// fewer narrow rows a deeper prefetch would exceed 256 VGPRs.
template <int NB, int NW>
__device__ __forceinline__ void lds_solve(const double* __restrict__ F, double* col) {
    constexpr int PF = NW >= NB - 9 ? 5 : 3;  // narrow rows leave registers for a deeper prefetch
    double2 L[PF][4];
    double nb[PF];  // col[i + 8] for the coming rows
#pragma unroll
    for (int p = 0; p < PF; ++p) {
        const double2* f = reinterpret_cast<const double2*>(F + p * FACW);
#pragma unroll
        for (int j = 0; j < (p < NW ? 2 : 4); ++j) L[p][j] = f[j];
        nb[p] = 8 + p < NB ? col[2 * (8 + p)] : 0.0;
    }
    double b0 = col[0], b1 = col[2], b2 = col[4], b3 = col[6];
    double b4 = col[8], b5 = col[10], b6 = col[12], b7 = col[14];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int p = i % PF;
        const double2 l01 = L[p][0], l23 = L[p][1], l45 = L[p][2], l67 = L[p][3];
        const double next = nb[p];
        if (i + PF < NB) {
            const double2* f = reinterpret_cast<const double2*>(F + (i + PF) * FACW);
#pragma unroll
            for (int j = 0; j < (i + PF < NW ? 2 : 4); ++j) L[p][j] = f[j];
            nb[p] = i + PF + 8 < NB ? col[2 * (i + PF + 8)] : 0.0;
        }
        const double y = b0;
        col[2 * i] = y;
        b0 = b1 - l01.x * y;
        b1 = b2 - l01.y * y;
        b2 = b3 - l23.x * y;
        b3 = b4 - l23.y * y;
        if (i < NW) {
            b4 = b5;
            b5 = b6;
            b6 = b7;
            b7 = next;
        } else {
            b4 = b5 - l45.x * y;
            b5 = b6 - l45.y * y;
            b6 = b7 - l67.x * y;
            b7 = next - l67.y * y;
        }
    }
    double2 U[PF][3];  // (u1, u2), (u3, u4), (1/U_ii, pad)
    double nc[PF];     // col[i - 4] for the coming rows
#pragma unroll
    for (int p = 0; p < PF; ++p) {
        const int i = NB - 1 - p;
        const double2* f = reinterpret_cast<const double2*>(F + i * FACW + 8);
#pragma unroll
        for (int j = 0; j < 3; ++j) U[p][j] = f[j];
        nc[p] = i - 4 >= 0 ? col[2 * (i - 4)] : 0.0;
    }
    double c0 = col[2 * (NB - 1)], c1 = col[2 * (NB - 2)], c2 = col[2 * (NB - 3)], c3 = col[2 * (NB - 4)];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int i = NB - 1 - t, p = t % PF;
        const double2 u12 = U[p][0], u34 = U[p][1], dv = U[p][2];
        const double next = nc[p];
        if (t + PF < NB) {
            const double2* f = reinterpret_cast<const double2*>(F + (i - PF) * FACW + 8);
#pragma unroll
            for (int j = 0; j < 3; ++j) U[p][j] = f[j];
            nc[p] = i - PF - 4 >= 0 ? col[2 * (i - PF - 4)] : 0.0;
        }
        const double x = c0 * dv.x;
        col[2 * i] = x;
        c0 = c1 - u12.x * x;
        c1 = c2 - u12.y * x;
        c2 = c3 - u34.x * x;
        c3 = next - u34.y * x;
    }
}

// Factors moving from global memory to LDS in two halves: load() issues all
// 16-byte loads of this thread into registers (branch-free, clamped
// indices), store() writes them into FACW-double row records at stride FS
// doubles and zeroes rows N..NB-1.  Factor f has global index base + f *
// stride.  A factor's main records (5 double2 per row) are copied whole, its
// tail records (2 double2 per row) from row NW on: the narrow rows before NW
// never read their tail, whose LDS slots are left as they are.
template <int NB, int NFMAX, int NTHR, int NW>
struct FactorStage {
    static constexpr int M2 = FMAIN / 2, T2 = FTAIL / 2, R2 = FACW / 2;
    static constexpr int MAXIT = (NFMAX * (NB * M2 + (NB - NW) * T2) + NTHR - 1) / NTHR;
    double2 tmp[MAXIT];
    // double2 r of a factor's copied part: offset in its HBM block, offset in LDS
    __device__ __forceinline__ static int src(int r, int N) { return r < N * M2 ? r : r + NW * T2; }
    __device__ __forceinline__ static int dst(int r, int N) {
        if (r < N * M2) {
            const int i = r / M2, s = r % M2;
            return i * R2 + (s < 2 ? s : s + T2);  // L[1..4] -> slots 0, 1; U, 1/U -> 4, 5, 6
        }
        const int t = r - N * M2;
        return (NW + t / T2) * R2 + 2 + t % T2;  // L[5..8] -> slots 2, 3
    }
    __device__ __forceinline__ void load(const double* fac, size_t base, size_t stride, int nf, int N, int t) {
        const int per = N * M2 + (N - NW) * T2, total = nf * per;
        const size_t FSZ = (size_t)N * FACW;
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) {
            const int e = min(t + it * NTHR, total - 1);
            tmp[it] = reinterpret_cast<const double2*>(fac + (base + (e / per) * stride) * FSZ)[src(e % per, N)];
        }
    }
    __device__ __forceinline__ void store(double* sF, int FS, int nf, int N, int t) const {
        const int per = N * M2 + (N - NW) * T2, total = nf * per;
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) {
            const int e = t + it * NTHR;
            if (e < total) reinterpret_cast<double2*>(sF + (e / per) * FS)[dst(e % per, N)] = tmp[it];
        }
        const int zper = (NB - N) * FACW;
        for (int e = t; e < nf * zper; e += NTHR) sF[(e / zper) * FS + N * FACW + e % zper] = 0.0;
    }
};

constexpr int NSLOT = 8;     // modes per workgroup: up to 4 values of m, both signs of k

// One workgroup = 4 waves handles |k| = kabs and GM consecutive m
// (GM = 4, 2, 1 for mp = 1, 2, >= 3 so that the Helmholtz wavenumbers
// mp*m-1 .. mp*m+1 of the block form one contiguous range of <= 6 values,
// shared between neighbouring m).  Slot q = 2 j + s is mode (m0 + j, s ? -k : +k).
// Wave w does the radial-line work of slots 2w, 2w+1; wave 0 does the
// substitutions with one lane per real right-hand side.
__device__ __forceinline__ void vort_row_w(const RowW& w1, double rinv, int s0, int n, int m, double kap,
                                           const dcplx* up, const dcplx* um, const dcplx* uz,
                                           dcplx& wp, dcplx& wm, dcplx& wz) {
    const int pe = m & 1, po = (m + 1) & 1;
    const dcplx duz = w1.apply(pe, uz, s0);
    const dcplx dup = w1.apply(po, up, s0);
    const dcplx dum = w1.apply(po, um, s0);
    const dcplx imz = (double(m) * rinv) * ix(uz[n]);
    wp = imz - ix(duz) - kap * up[n];
    wm = imz + ix(duz) + kap * um[n];
    const dcplx ap = dup + (double(1 + m) * rinv) * up[n];
    const dcplx am = dum + (double(1 - m) * rinv) * um[n];
    wz = 0.5 * ix(am - ap);
}

template <typename TNL, int NB, int NW>
__device__ __forceinline__ void k_solve_body(const SolveArgs& a) {
    constexpr int FS = NB * FACW + 4;  // factor stride (doubles): spreads LDS banks
    constexpr int XS = NB + 1;         // radial line stride (complex)
    __shared__ __align__(16) double sF[NFH * FS];
    __shared__ __align__(16) dcplx sX[NSLOT][3][XS];
    __shared__ dcplx sY[NSLOT][XS];
    __shared__ dcplx sA[NSLOT][4];
    __shared__ double sGam;
    dcplx(*sU)[3][XS] = reinterpret_cast<dcplx(*)[3][XS]>(sF);  // u^n staging (aliases factors)

    const Tables& t = a.t;
    const int N = a.N, K = a.K, nk = a.nk, mp = a.mp;
    const int GM = a.gm;
    const int nblk = (a.M + GM - 1) / GM;
    // Consecutive block indices go round-robin to the 8 XCDs; each XCD takes
    // a contiguous range of tiles instead, so the m-blocks of one |k|, which
    // share Helmholtz factors, meet in its L2.
    const int ntiles = (int)gridDim.x;
    const int tile = ntiles % 8 == 0 ? (blockIdx.x % 8) * (ntiles / 8) + blockIdx.x / 8 : (int)blockIdx.x;
    const int kabs = tile / nblk;
    const int m0 = (tile % nblk) * GM;
    const int tid = threadIdx.x, n = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
    const size_t S = (size_t)a.M * nk * N;
    const int mu_lo = max(mp * m0 - 1, 0);
    const int nr = n < N ? n : N - 1;  // lanes past the last row read a valid row
    RowW W1;  // first-derivative weights of this lane's row, both parities
    W1.load(t.d1, N, nr);
    const int s0r = t.s0[nr];
    const double rinvr = t.rinv[nr];

    const int nfp = min(GM, a.M - m0);
    const int mu_hi = min(mp * (m0 + GM - 1) + 1, a.MU - 1);
    const int nfh = mu_hi - mu_lo + 1;

    auto slot_ok = [&](int q) {
        const int j = q >> 1, s = q & 1, mi = m0 + j;
        return j < GM && mi < a.M && (s == 0 || (kabs > 0 && mi > 0));
    };
    auto slot_k = [&](int q) { return (q & 1) ? -kabs : kabs; };
    auto slot_off = [&](int q) {  // offset of row 0 of slot q in one field
        return ((size_t)(m0 + (q >> 1)) * nk + (slot_k(q) + K - 1)) * N;
    };

    // rows N..NB-1 of the line buffers stay zero (branch-free substitution)
    for (int i = tid; i < NSLOT * (NB + 1 - N); i += 256) {
        const int q = i / (NB + 1 - N), r = N + i % (NB + 1 - N);
        sY[q][r] = dcplx{0.0, 0.0};
        sX[q][0][r] = sX[q][1][r] = sX[q][2][r] = dcplx{0.0, 0.0};
    }
    // ---- load u^n (or R) of this wave's slots ---------------------------
    for (int q = 2 * w; q < 2 * w + 2; ++q) {
        if (!slot_ok(q) || n >= N) continue;
        const size_t off = slot_off(q) + n;
        if (a.kind == OPF_SOLVE_RAW) {
            const dcplx rr = load_c<double>(a.n0, off), rt = load_c<double>(a.n0, S + off);
            sX[q][0][n] = rr + ix(rt);
            sX[q][1][n] = rr - ix(rt);
            sX[q][2][n] = load_c<double>(a.n0, 2 * S + off);
        } else {
            const dcplx ur = load_c<double>(a.u0, off), ut = load_c<double>(a.u0, S + off);
            sU[q][0][n] = ur + ix(ut);
            sU[q][1][n] = ur - ix(ut);
            sU[q][2][n] = load_c<double>(a.u0, 2 * S + off);
        }
    }
    __syncthreads();

    // ---- R = [1/dt + (1-c) L / Re] u^n + N (+ forcing) --------------------
    if (a.kind != OPF_SOLVE_RAW && n < N) {
        const int s0 = s0r;
        const double rinv = rinvr;
        RowW W2;  // second-derivative weights, needed here only
        W2.load(t.d2, N, n);
        for (int q = 2 * w; q < 2 * w + 2; ++q) {
            if (!slot_ok(q)) continue;
            const int m = mp * (m0 + (q >> 1)), k = slot_k(q);
            const double kap2 = a.alpha * k * a.alpha * k;
            const size_t off = slot_off(q) + n;
            dcplx nr, nt, nz;
            if (a.kind == OPF_SOLVE_PRED) {
                nr = load_c<TNL>(a.n0, off);
                nt = load_c<TNL>(a.n0, S + off);
                nz = load_c<TNL>(a.n0, 2 * S + off);
            } else {
                const double cc = a.c, c1 = 1.0 - a.c;
                nr = c1 * load_c<TNL>(a.n0, off) + cc * load_c<TNL>(a.n1, off);
                nt = c1 * load_c<TNL>(a.n0, S + off) + cc * load_c<TNL>(a.n1, S + off);
                nz = c1 * load_c<TNL>(a.n0, 2 * S + off) + cc * load_c<TNL>(a.n1, 2 * S + off);
            }
            const dcplx nl[3] = {nr + ix(nt), nr - ix(nt), nz};
            const int mus[3] = {m + 1, m - 1, m};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int mu = mus[c], p = abs(mu) & 1;
                const dcplx* line = sU[q][c];
                const dcplx d2 = W2.apply(p, line, s0);
                const dcplx d1 = W1.apply(p, line, s0);
                const double diag = double(mu) * double(mu) * rinv * rinv + kap2;
                const dcplx Lu = d2 + rinv * d1 - diag * line[n];
                sX[q][c][n] = a.inv_dt * line[n] + a.aexp * Lu + nl[c];
            }
            if (m == 0 && k == 0) sX[q][2][n].x += a.force;
        }
    }
    __syncthreads();

    // ---- pressure-Poisson right-hand side div R (P(1) = 0); stage L factors
    {  // pressure factors L_{m,|k|}, m0 <= m < m0 + GM (the u^n staging area is free now)
        FactorStage<NB, 4, 256, NW> ppe;
        ppe.load(t.fac, (size_t)a.MU * K + (size_t)m0 * K + kabs, K, nfp, N, tid);
        ppe.store(sF, FS, nfp, N, tid);
    }
    if (n < N) {
        const int s0 = s0r;
        const double rinv = rinvr;
        for (int q = 2 * w; q < 2 * w + 2; ++q) {
            if (!slot_ok(q)) continue;
            const int m = mp * (m0 + (q >> 1));
            const double kap = a.alpha * slot_k(q);
            const int po = (m + 1) & 1;
            dcplx d = {0.0, 0.0};
            if (n < N - 1 && !(m == 0 && kap == 0.0)) {
                const dcplx ap = W1.apply(po, sX[q][0], s0) + (double(1 + m) * rinv) * sX[q][0][n];
                const dcplx am = W1.apply(po, sX[q][1], s0) + (double(1 - m) * rinv) * sX[q][1][n];
                d = 0.5 * (ap + am) + kap * ix(sX[q][2][n]);
            }
            sY[q][n] = d;
        }
    }
    __syncthreads();
    if (w == 0 && n < 2 * NSLOT) {
        const int q = n >> 1;
        if (slot_ok(q)) lds_solve<NB, NW>(sF + (q >> 1) * FS, &sY[q][0].x + (n & 1));
    }
    __syncthreads();

    // ---- R -= grad P; (0,0): u_r = 0, real R_theta and R_z; stage H factors
    {  // Helmholtz factors H_{mu,|k|}, mu_lo <= mu <= mu_hi
        FactorStage<NB, NFH, 256, NW> helm;
        helm.load(t.fac, (size_t)mu_lo * K + kabs, K, nfh, N, tid);
        helm.store(sF, FS, nfh, N, tid);
    }
    if (n < N) {
        const int s0 = s0r;
        const double rinv = rinvr;
        for (int q = 2 * w; q < 2 * w + 2; ++q) {
            if (!slot_ok(q)) continue;
            const int m = mp * (m0 + (q >> 1));
            const double kap = a.alpha * slot_k(q);
            if (n == N - 1) {
                sX[q][0][n] = sX[q][1][n] = sX[q][2][n] = dcplx{0.0, 0.0};
                if (m == 0 && kap == 0.0 && a.wall) {  // (0,0): Dirichlet values u_theta(1), u_z(1)
                    const size_t w0 = (size_t)(K - 1) * 2, ws = (size_t)a.M * nk * 2;
                    sX[q][0][n] = dcplx{a.wall[ws + w0], 0.0};
                    sX[q][2][n] = dcplx{a.wall[2 * ws + w0], 0.0};
                }
            } else if (m == 0 && kap == 0.0) {
                const dcplx d = sX[q][0][n] - sX[q][1][n];  // 2 i R_theta
                sX[q][0][n] = dcplx{0.5 * d.y, 0.0};
                sX[q][1][n] = dcplx{0.0, 0.0};
                sX[q][2][n] = dcplx{sX[q][2][n].x, 0.0};
            } else {
                const dcplx dP = W1.apply(m & 1, sY[q], s0);
                const dcplx mP = (double(m) * rinv) * sY[q][n];
                sX[q][0][n] = sX[q][0][n] - (dP - mP);
                sX[q][1][n] = sX[q][1][n] - (dP + mP);
                sX[q][2][n] = sX[q][2][n] - kap * ix(sY[q][n]);
            }
        }
    }
    __syncthreads();
    if (w == 0 && n < 6 * NSLOT) {
        const int q = n / 6, c = (n >> 1) % 3;
        if (slot_ok(q)) {
            const int m = mp * (m0 + (q >> 1));
            const int mu = c == 0 ? m + 1 : (c == 1 ? abs(m - 1) : m);
            lds_solve<NB, NW>(sF + (mu - mu_lo) * FS, &sX[q][c][0].x + (n & 1));
        }
    }
    __syncthreads();

    // ---- influence matrix a = -A^{-1} g(u_b); fixed flux on (0,0) --------
    // The influence data of this wave's m (one radial row per lane) is loaded
    // now, so its latency overlaps the influence step of the first lanes.
    double hv[NHOM];
    {
        const double* h = t.hom + ((size_t)min(m0 + w, a.M - 1) * K + kabs) * NHOM * N;
#pragma unroll
        for (int j = 0; j < NHOM; ++j) hv[j] = h[j * N + nr];
    }
    if (tid < NSLOT && slot_ok(tid)) {
        const int q = tid;
        const int mi = m0 + (q >> 1), m = mp * mi, k = slot_k(q);
        if (m == 0 && k == 0) {
            double qs = 0.0;
            for (int i = 0; i < N; ++i) qs += t.quad[i] * sX[q][2][i].x;
            const double gamma = a.fixed_flux ? (0.25 - qs) * t.qG_inv : 0.0;
            sGam = gamma;
            if (a.beta_out) *a.beta_out = gamma * a.Re * 0.25;
        } else {
            const double kap = a.alpha * k;
            const int e = N - 1, s0 = t.s0[e];
            const double rinv = t.rinv[e];
            const double* w1 = t.d1 + (((m + 1) & 1) * N + e) * W9;
            const dcplx ap = stencil(w1, sX[q][0], s0) + (double(1 + m) * rinv) * sX[q][0][e];
            const dcplx am = stencil(w1, sX[q][1], s0) + (double(1 - m) * rinv) * sX[q][1][e];
            dcplx g[4] = {sX[q][0][e], sX[q][1][e], sX[q][2][e], 0.5 * (ap + am) + kap * ix(sX[q][2][e])};
            if (a.wall) {  // drive g to the wall velocity (b_r +- i b_theta, b_z, 0) instead of 0
                const size_t wi = ((size_t)mi * nk + (k + K - 1)) * 2, ws = (size_t)a.M * nk * 2;
                const dcplx br = {a.wall[wi], a.wall[wi + 1]}, bt = {a.wall[ws + wi], a.wall[ws + wi + 1]};
                g[0] = g[0] - (br + ix(bt));
                g[1] = g[1] - (br - ix(bt));
                g[2] = g[2] - dcplx{a.wall[2 * ws + wi], a.wall[2 * ws + wi + 1]};
            }
            const double* A = t.ainv + (((size_t)mi * nk + (k + K - 1)) * 16) * 2;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dcplx acc = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc = acc + cm(dcplx{A[2 * (4 * i + j)], A[2 * (4 * i + j) + 1]}, g[j]);
                sA[q][i] = dcplx{-acc.x, -acc.y};
            }
        }
    }
    __syncthreads();
    if (n < N) {
        for (int q = 2 * w; q < 2 * w + 2; ++q) {
            if (!slot_ok(q)) continue;
            const int mi = m0 + (q >> 1), m = mp * mi, k = slot_k(q);
            if (m == 0 && k == 0) {
                const double ut = sX[q][0][n].x;
                const double uz = sX[q][2][n].x + sGam * t.green[n];
                sX[q][0][n] = dcplx{0.0, ut};
                sX[q][1][n] = dcplx{0.0, -ut};
                sX[q][2][n] = dcplx{uz, 0.0};
                sY[q][n] = dcplx{0.0, 0.0};
            } else {
                const double kap = a.alpha * k;
                const double h1p = hv[0], h1m = hv[1], qv = hv[2], h2 = hv[3], h3 = hv[4], h4 = hv[5], P1 = hv[6];
                const dcplx a1 = sA[q][0], a2 = sA[q][1], a3 = sA[q][2], a4 = sA[q][3];
                sX[q][0][n] = sX[q][0][n] + h1p * a1 + h2 * a2;
                sX[q][1][n] = sX[q][1][n] + h1m * a1 + h3 * a3;
                sX[q][2][n] = sX[q][2][n] - (kap * qv) * ix(a1) + h4 * a4;  // h1: u_z = -i kappa q
                sY[q][n] = sY[q][n] + P1 * a1;
            }
        }
    }
    __syncthreads();

    // ---- output u (r, theta, z); omega from the stored components --------
    // omega is computed from (u_r, u_theta, u_z) as stored, so it equals what
    // the standalone vorticity kernel gives for the same state.
    if (n < N) {
        for (int q = 2 * w; q < 2 * w + 2; ++q) {
            if (!slot_ok(q)) continue;
            const int mi = m0 + (q >> 1);
            const bool mirror = (mi == 0 && kabs > 0);  // m = 0: -k is the conjugate of +k
            const dcplx up = sX[q][0][n], um = sX[q][1][n], uz = sX[q][2][n];
            const dcplx ur = 0.5 * (up + um), ut = 0.5 * dcplx{(up - um).y, -(up - um).x};
            const dcplx uo[3] = {ur, ut, uz};
            const size_t off = slot_off(q) + n;
            const size_t offc = ((size_t)mi * nk + (K - 1 - kabs)) * N + n;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const dcplx uc = {uo[c].x, -uo[c].y};
                if (a.u_out) {
                    store_c<double>(a.u_out, c * S + off, uo[c]);
                    if (mirror) store_c<double>(a.u_out, c * S + offc, uc);
                }
                if (a.u_out32) {
                    store_c<float>(a.u_out32, c * S + off, uo[c]);
                    if (mirror) store_c<float>(a.u_out32, c * S + offc, uc);
                }
            }
            if (a.p_out) {
                const dcplx pp = sY[q][n];
                store_c<double>(a.p_out, off, pp);
                if (mirror) store_c<double>(a.p_out, offc, dcplx{pp.x, -pp.y});
            }
            sX[q][0][n] = ur + ix(ut);
            sX[q][1][n] = ur - ix(ut);
        }
    }
    __syncthreads();
    if (a.w_out && n < N) {
        for (int q = 2 * w; q < 2 * w + 2; ++q) {
            if (!slot_ok(q)) continue;
            const int mi = m0 + (q >> 1), m = mp * mi, k = slot_k(q);
            const bool mirror = (mi == 0 && kabs > 0);
            dcplx wp, wm, wz;
            vort_row_w(W1, rinvr, s0r, n, m, a.alpha * k, sX[q][0], sX[q][1], sX[q][2], wp, wm, wz);
            const dcplx wo[3] = {0.5 * (wp + wm), 0.5 * dcplx{(wp - wm).y, -(wp - wm).x}, wz};
            const size_t off = slot_off(q) + n;
            const size_t offc = ((size_t)mi * nk + (K - 1 - kabs)) * N + n;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                store_c<TNL>(a.w_out, c * S + off, wo[c]);
                if (mirror) store_c<TNL>(a.w_out, c * S + offc, dcplx{wo[c].x, -wo[c].y});
            }
        }
    }
}

template <typename TNL, int NB, int NW>
__global__ __launch_bounds__(256) void k_solve(SolveArgs a) { k_solve_body<TNL, NB, NW>(a); }
template <typename TNL, int NB, int NW>
__global__ __launch_bounds__(256) void k_solve_b(const SolveArgs* __restrict__ aa) {
    // the member's record is read in place (a private copy would live in scratch)
    k_solve_body<TNL, NB, NW>(aa[blockIdx.y]);
}

// Standalone vorticity of an external-layout state.  With a.mirror set
// (states, which are real fields) the m = 0, k < 0 modes are written as the
// conjugates of k > 0, as the solve kernel does; otherwise every mode is
// computed on its own.
__global__ __launch_bounds__(64) void k_vorticity(AuxArgs a) {
    __shared__ dcplx sL[3][LSTR];
    const int N = a.N, K = a.K, nk = a.nk;
    const int mi = blockIdx.x / nk, kk = blockIdx.x % nk;
    if (a.mirror && mi == 0 && kk < K - 1) return;
    const int m = a.mp * mi, n = threadIdx.x;
    const size_t S = (size_t)a.M * nk * N;
    const size_t off = ((size_t)mi * nk + kk) * N + n;
    if (n < N) {
        const dcplx ur = load_c<double>(a.u, off), ut = load_c<double>(a.u, S + off);
        sL[0][n] = ur + ix(ut);
        sL[1][n] = ur - ix(ut);
        sL[2][n] = load_c<double>(a.u, 2 * S + off);
    }
    __syncthreads();
    if (n < N) {
        dcplx wp, wm, wz;
        vort_row(a.t, N, n, m, a.alpha * (kk - (K - 1)), sL[0], sL[1], sL[2], wp, wm, wz);
        const dcplx wo[3] = {0.5 * (wp + wm), 0.5 * dcplx{(wp - wm).y, -(wp - wm).x}, wz};
        const bool mirror = a.mirror && mi == 0 && kk > K - 1;
        const size_t offc = ((size_t)mi * nk + (2 * (K - 1) - kk)) * N + n;
        for (int c = 0; c < 3; ++c) {
            store_c<double>(a.w, c * S + off, wo[c]);
            if (mirror) store_c<double>(a.w, c * S + offc, dcplx{wo[c].x, -wo[c].y});
        }
    }
}

// Per-m quadrature sums of |u|^2 and |omega|^2 over k and the three
// components (diagnostics); fixed summation order.
__global__ __launch_bounds__(256) void k_energy(AuxArgs a) {
    __shared__ double s_u[256], s_w[256];
    const int N = a.N, nk = a.nk, mi = blockIdx.x;
    const size_t S = (size_t)a.M * nk * N;
    double eu = 0.0, ew = 0.0;
    for (int i = threadIdx.x; i < nk * N; i += 256) {
        const int n = i % N;
        const size_t off = (size_t)mi * nk * N + i;
        double su = 0.0, sw = 0.0;
        for (int c = 0; c < 3; ++c) {
            const dcplx u = load_c<double>(a.u, c * S + off);
            const dcplx w = load_c<double>(a.w, c * S + off);
            su += u.x * u.x + u.y * u.y;
            sw += w.x * w.x + w.y * w.y;
        }
        eu += a.t.quad[n] * su;
        ew += a.t.quad[n] * sw;
    }
    s_u[threadIdx.x] = eu;
    s_w[threadIdx.x] = ew;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s_u[threadIdx.x] += s_u[threadIdx.x + h];
            s_w[threadIdx.x] += s_w[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partial[2 * mi] = s_u[0];
        a.partial[2 * mi + 1] = s_w[0];
    }
}

int default_gm(int mp) { return mp == 1 ? 4 : (mp <= 3 ? 2 : 1); }

bool gm_ok(int gm, int mp) { return gm >= 1 && gm <= 4 && mp * (gm - 1) + 3 <= NFH; }

hipError_t launch_solve_batch(const SolveArgs& a, const SolveArgs* batch, int members, int precision,
                              hipStream_t s) {
    const bool b = batch != nullptr;
    const dim3 grid(a.K * ((a.M + a.gm - 1) / a.gm), b ? members : 1), block(256);
    // narrow-window rows: the largest compiled count that a.narrow allows
    // (NB - 9 when N = NB, NB - 25 when N >= NB - 16, else none); the members
    // of a batch share N and with it narrow
#define OPF_SOLVE_LAUNCH(TNL, NB, NW)                                                   \
    if (b) hipLaunchKernelGGL((k_solve_b<TNL, NB, NW>), grid, block, 0, s, batch); \
    else hipLaunchKernelGGL((k_solve<TNL, NB, NW>), grid, block, 0, s, a);
#define OPF_SOLVE_NW(TNL, NB)                                                       \
    if (a.narrow >= NB - 9) { OPF_SOLVE_LAUNCH(TNL, NB, NB - 9) }                 \
    else if (a.narrow >= NB - 25) { OPF_SOLVE_LAUNCH(TNL, NB, NB - 25) }          \
    else { OPF_SOLVE_LAUNCH(TNL, NB, 0) }
    if (a.N <= 32) {
        if (precision == OPF_MIXED) { OPF_SOLVE_NW(float, 32) }
        else { OPF_SOLVE_NW(double, 32) }
    } else if (a.N <= 48) {
        if (precision == OPF_MIXED) { OPF_SOLVE_NW(float, 48) }
        else { OPF_SOLVE_NW(double, 48) }
    } else {
        if (precision == OPF_MIXED) { OPF_SOLVE_NW(float, 64) }
        else { OPF_SOLVE_NW(double, 64) }
    }
#undef OPF_SOLVE_NW
#undef OPF_SOLVE_LAUNCH
    return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, int precision, hipStream_t s) {
    return launch_solve_batch(a, nullptr, 1, precision, s);
}

// Boundary-condition residual and interior divergence of every mode (one
// 64-lane workgroup per mode, lanes = radial nodes), in the (+,-,z) form
// (u+- = u_r +- i u_theta): div u = (1/2)[u+' + (1+m) u+/r]
// + (1/2)[u-' + (1-m) u-/r] + i kappa u_z.  part[2q] = max(|u+(1)|, |u-(1)|,
// |u_z(1)|, |div u(1)|), part[2q+1] = max over n < N-1 of |div u(r_n)|.
__global__ __launch_bounds__(64) void k_divg(AuxArgs a, double* __restrict__ part) {
    __shared__ dcplx sL[3][LSTR];
    const int N = a.N, K = a.K, nk = a.nk;
    const int q = blockIdx.x, mi = q / nk, kk = q % nk;
    const int m = a.mp * mi, n = threadIdx.x;
    const double kap = a.alpha * (kk - (K - 1));
    const size_t S = (size_t)a.M * nk * N;
    const size_t off = (size_t)q * N + n;
    if (n < N) {
        const dcplx ur = load_c<double>(a.u, off), ut = load_c<double>(a.u, S + off);
        sL[0][n] = ur + ix(ut);
        sL[1][n] = ur - ix(ut);
        sL[2][n] = load_c<double>(a.u, 2 * S + off);
    }
    __syncthreads();
    double gv = 0.0, dv = 0.0;
    if (n < N) {
        const int s0 = a.t.s0[n];
        const double rinv = a.t.rinv[n];
        const double* w1 = a.t.d1 + (((m + 1) & 1) * N + n) * W9;
        const dcplx up = sL[0][n], um = sL[1][n], uz = sL[2][n];
        const dcplx ap = stencil(w1, sL[0], s0) + (double(1 + m) * rinv) * up;
        const dcplx am = stencil(w1, sL[1], s0) + (double(1 - m) * rinv) * um;
        const dcplx d = 0.5 * (ap + am) + kap * ix(uz);
        const double ad = sqrt(d.x * d.x + d.y * d.y);
        if (n == N - 1) {
            dcplx bp = {0.0, 0.0}, bm = {0.0, 0.0}, bz = {0.0, 0.0};
            if (a.wall) {  // residual against the wall velocity
                const size_t wi = (size_t)q * 2, ws = (size_t)a.M * nk * 2;
                const dcplx br = {a.wall[wi], a.wall[wi + 1]}, bt = {a.wall[ws + wi], a.wall[ws + wi + 1]};
                bp = br + ix(bt);
                bm = br - ix(bt);
                bz = dcplx{a.wall[2 * ws + wi], a.wall[2 * ws + wi + 1]};
            }
            const dcplx ep = up - bp, em = um - bm, ez = uz - bz;
            const double a1 = sqrt(ep.x * ep.x + ep.y * ep.y), a2 = sqrt(em.x * em.x + em.y * em.y);
            const double a3 = sqrt(ez.x * ez.x + ez.y * ez.y);
            gv = fmax(fmax(a1, a2), fmax(a3, ad));
        } else {
            dv = ad;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        gv = fmax(gv, __shfl_xor(gv, o, 64));
        dv = fmax(dv, __shfl_xor(dv, o, 64));
    }
    if (n == 0) {
        part[2 * q] = gv;
        part[2 * q + 1] = dv;
    }
}

hipError_t launch_divg(const AuxArgs& a, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_divg, dim3(a.M * a.nk), dim3(64), 0, s, a, part);
    return hipGetLastError();
}

hipError_t launch_vorticity(const AuxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_vorticity, dim3(a.M * a.nk), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_energy(const AuxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_energy, dim3(a.M), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace opf
