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
// One 64-lane workgroup handles the mode pair (m, +k), (m, -k): both use
// the same four factors (they depend on |k|).  Lanes are radial nodes for
// the stencil work; for the substitutions each lane owns one real
// right-hand side (a real or imaginary part of one component of one mode)
// and walks the rows with the factor staged in LDS.  m = 0 solves k >= 0
// only and writes the conjugate into -k (Hermitian symmetry of a real
// field); mode (0,0) has u_r = 0, no pressure and the fixed-flux correction.
#include "opf_internal.h"

namespace opf {

constexpr int LSTR = NMAX + 2;            // LDS line stride (complex): avoids bank aliasing
constexpr int FSTR = NMAX * FACW + 2;     // LDS factor stride (doubles)

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

// Solve A x = b in place for one real right-hand side (element i at v[2*i]),
// A = LU without pivoting; factor row i: F[0..7] multiply x[i-1..i-8] in the
// forward pass, F[8..11] multiply x[i+1..i+4] in the backward pass,
// F[12] = 1 / U_ii.  Out-of-band entries are zero.
__device__ __forceinline__ void lu_solve(const double* F, double* v, int N) {
    double w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0, w6 = 0, w7 = 0;
    for (int i = 0; i < N; ++i) {
        const double* f = F + i * FACW;
        double acc = v[2 * i];
        acc -= f[7] * w7;
        acc -= f[6] * w6;
        acc -= f[5] * w5;
        acc -= f[4] * w4;
        acc -= f[3] * w3;
        acc -= f[2] * w2;
        acc -= f[1] * w1;
        acc -= f[0] * w0;
        v[2 * i] = acc;
        w7 = w6; w6 = w5; w5 = w4; w4 = w3; w3 = w2; w2 = w1; w1 = w0; w0 = acc;
    }
    double x0 = 0, x1 = 0, x2 = 0, x3 = 0;
    for (int i = N - 1; i >= 0; --i) {
        const double* f = F + i * FACW;
        double acc = v[2 * i];
        acc -= f[11] * x3;
        acc -= f[10] * x2;
        acc -= f[9] * x1;
        acc -= f[8] * x0;
        acc *= f[12];
        v[2 * i] = acc;
        x3 = x2; x2 = x1; x1 = x0; x0 = acc;
    }
}

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

template <typename TNL>
__global__ __launch_bounds__(64) void k_solve(SolveArgs a) {
    __shared__ dcplx sU[2][3][LSTR];  // u^n (+,-,z)
    __shared__ dcplx sR[2][3][LSTR];  // right-hand side -> solution
    __shared__ dcplx sP[2][LSTR];     // div R -> pressure
    __shared__ double sF[3][FSTR];    // LU factors
    __shared__ dcplx sA[2][4];        // influence coefficients a_j
    __shared__ double sRed[64];

    const Tables& t = a.t;
    const int N = a.N, K = a.K, nk = a.nk;
    const int mi = blockIdx.x / K, kabs = blockIdx.x % K;
    const int m = a.mp * mi;
    const bool zero_mode = (mi == 0 && kabs == 0);
    const int nsig = (mi > 0 && kabs > 0) ? 2 : 1;
    const int tid = threadIdx.x;
    const int n = tid;
    const size_t S = (size_t)a.M * nk * N;                 // one field
    const int hp = abs(m + 1), hm = abs(m - 1), hz = m;    // Helmholtz |mu|
    const size_t FSZ = (size_t)N * FACW;

    // ---- stage the pressure factor; load u^n or R -----------------------
    if (!zero_mode) {
        const double* src = t.fac + ((size_t)a.MU * K + (size_t)mi * K + kabs) * FSZ;
        for (int i = tid; i < N * FACW; i += 64) sF[0][i] = src[i];
    }
    for (int s = 0; s < nsig; ++s) {
        const int kk = s == 0 ? K - 1 + kabs : K - 1 - kabs;
        const size_t off = ((size_t)mi * nk + kk) * N + n;
        if (n < N) {
            if (a.kind == OPF_SOLVE_RAW) {
                const dcplx rr = load_c<double>(a.n0, off), rt = load_c<double>(a.n0, S + off);
                sR[s][0][n] = rr + ix(rt);
                sR[s][1][n] = rr - ix(rt);
                sR[s][2][n] = load_c<double>(a.n0, 2 * S + off);
            } else {
                const dcplx ur = load_c<double>(a.u0, off), ut = load_c<double>(a.u0, S + off);
                sU[s][0][n] = ur + ix(ut);
                sU[s][1][n] = ur - ix(ut);
                sU[s][2][n] = load_c<double>(a.u0, 2 * S + off);
            }
        }
    }
    __syncthreads();

    // ---- right-hand side R = [1/dt + (1-c) L / Re] u^n + N (+ forcing) ----
    if (a.kind != OPF_SOLVE_RAW && n < N) {
        const int s0 = t.s0[n];
        const double rinv = t.rinv[n];
        for (int s = 0; s < nsig; ++s) {
            const int k = s == 0 ? kabs : -kabs;
            const double kap2 = a.alpha * k * a.alpha * k;
            const int kk = k + K - 1;
            const size_t off = ((size_t)mi * nk + kk) * N + n;
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
                const dcplx* line = sU[s][c];
                const dcplx d2 = stencil(t.d2 + (p * N + n) * W9, line, s0);
                const dcplx d1 = stencil(t.d1 + (p * N + n) * W9, line, s0);
                const double diag = double(mu) * double(mu) * rinv * rinv + kap2;
                const dcplx Lu = d2 + rinv * d1 - diag * line[n];
                sR[s][c][n] = a.inv_dt * line[n] + a.aexp * Lu + nl[c];
            }
            if (zero_mode) sR[s][2][n].x += a.force;
        }
    }
    __syncthreads();

    if (!zero_mode) {
        // ---- pressure-Poisson right-hand side: div R, P(1) = 0 -----------
        if (n < N) {
            const int s0 = t.s0[n];
            const double rinv = t.rinv[n];
            const double* w1 = t.d1 + (((m + 1) & 1) * N + n) * W9;
            for (int s = 0; s < nsig; ++s) {
                const double kap = a.alpha * (s == 0 ? kabs : -kabs);
                dcplx d = {0.0, 0.0};
                if (n < N - 1) {
                    const dcplx ap = stencil(w1, sR[s][0], s0) + (double(1 + m) * rinv) * sR[s][0][n];
                    const dcplx am = stencil(w1, sR[s][1], s0) + (double(1 - m) * rinv) * sR[s][1][n];
                    d = 0.5 * (ap + am) + kap * ix(sR[s][2][n]);
                }
                sP[s][n] = d;
            }
        }
        __syncthreads();
        if (tid < 2 * nsig) lu_solve(sF[0], &sP[tid >> 1][0].x + (tid & 1), N);
        __syncthreads();
        // ---- stage Helmholtz factors; R -= grad P --------------------------
        {
            const double* fp = t.fac + ((size_t)hp * K + kabs) * FSZ;
            const double* fm = t.fac + ((size_t)hm * K + kabs) * FSZ;
            const double* fz = t.fac + ((size_t)hz * K + kabs) * FSZ;
            for (int i = tid; i < N * FACW; i += 64) {
                sF[0][i] = fp[i];
                sF[1][i] = fm[i];
                sF[2][i] = fz[i];
            }
        }
        if (n < N) {
            const int s0 = t.s0[n];
            const double rinv = t.rinv[n];
            const double* w1 = t.d1 + ((m & 1) * N + n) * W9;
            for (int s = 0; s < nsig; ++s) {
                const double kap = a.alpha * (s == 0 ? kabs : -kabs);
                if (n < N - 1) {
                    const dcplx dP = stencil(w1, sP[s], s0);
                    const dcplx mP = (double(m) * rinv) * sP[s][n];
                    sR[s][0][n] = sR[s][0][n] - (dP - mP);
                    sR[s][1][n] = sR[s][1][n] - (dP + mP);
                    sR[s][2][n] = sR[s][2][n] - kap * ix(sP[s][n]);
                } else {
                    sR[s][0][n] = sR[s][1][n] = sR[s][2][n] = dcplx{0.0, 0.0};
                }
            }
        }
        __syncthreads();
        // ---- Helmholtz solves ----------------------------------------------
        if (tid < 6 * nsig) {
            const int s = tid / 6, c = (tid >> 1) % 3;
            lu_solve(sF[c], &sR[s][c][0].x + (tid & 1), N);
        }
        __syncthreads();
        // ---- influence matrix: a = -A^{-1} g(u_b) --------------------------
        if (tid < nsig) {
            const int s = tid;
            const int k = s == 0 ? kabs : -kabs;
            const double kap = a.alpha * k;
            const int e = N - 1, s0 = t.s0[e];
            const double rinv = t.rinv[e];
            const double* w1 = t.d1 + (((m + 1) & 1) * N + e) * W9;
            const dcplx ap = stencil(w1, sR[s][0], s0) + (double(1 + m) * rinv) * sR[s][0][e];
            const dcplx am = stencil(w1, sR[s][1], s0) + (double(1 - m) * rinv) * sR[s][1][e];
            dcplx g[4] = {sR[s][0][e], sR[s][1][e], sR[s][2][e], 0.5 * (ap + am) + kap * ix(sR[s][2][e])};
            const double* A = t.ainv + (((size_t)mi * nk + (k + K - 1)) * 16) * 2;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dcplx acc = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < 4; ++j) acc = acc + cm(dcplx{A[2 * (4 * i + j)], A[2 * (4 * i + j) + 1]}, g[j]);
                sA[s][i] = dcplx{-acc.x, -acc.y};
            }
        }
        __syncthreads();
        if (n < N) {
            const double* h = t.hom + ((size_t)mi * K + kabs) * NHOM * N;
            const double h1p = h[n], h1m = h[N + n], q = h[2 * N + n];
            const double h2 = h[3 * N + n], h3 = h[4 * N + n], h4 = h[5 * N + n], P1 = h[6 * N + n];
            for (int s = 0; s < nsig; ++s) {
                const double kap = a.alpha * (s == 0 ? kabs : -kabs);
                const dcplx a1 = sA[s][0], a2 = sA[s][1], a3 = sA[s][2], a4 = sA[s][3];
                sR[s][0][n] = sR[s][0][n] + h1p * a1 + h2 * a2;
                sR[s][1][n] = sR[s][1][n] + h1m * a1 + h3 * a3;
                // h1 has u_z = -i kappa q
                sR[s][2][n] = sR[s][2][n] - (kap * q) * ix(a1) + h4 * a4;
                sP[s][n] = sP[s][n] + P1 * a1;
            }
        }
    } else {
        // ---- mode (0,0): u_r = 0; H_1 u_t = R_t; H_0 u_z = R_z + gamma -------
        {
            const double* f1 = t.fac + ((size_t)1 * K) * FSZ;
            const double* f0 = t.fac;
            for (int i = tid; i < N * FACW; i += 64) {
                sF[0][i] = f1[i];
                sF[2][i] = f0[i];
            }
        }
        if (n < N) {
            const dcplx d = sR[0][0][n] - sR[0][1][n];  // 2 i R_t
            const bool wall = n == N - 1;
            sR[0][0][n] = dcplx{wall ? 0.0 : 0.5 * d.y, 0.0};
            sR[0][2][n] = dcplx{wall ? 0.0 : sR[0][2][n].x, 0.0};
        }
        __syncthreads();
        if (tid == 0) lu_solve(sF[0], &sR[0][0][0].x, N);
        if (tid == 1) lu_solve(sF[2], &sR[0][2][0].x, N);
        __syncthreads();
        sRed[tid] = n < N ? t.quad[n] * sR[0][2][n].x : 0.0;
        __syncthreads();
        if (tid == 0) {
            double q = 0.0;
            for (int i = 0; i < N; ++i) q += sRed[i];
            const double gamma = a.fixed_flux ? (0.25 - q) * t.qG_inv : 0.0;
            sA[0][0] = dcplx{gamma, 0.0};
            if (a.beta_out) *a.beta_out = gamma * a.Re * 0.25;
        }
        __syncthreads();
        if (n < N) {
            const double ut = sR[0][0][n].x;
            const double uz = sR[0][2][n].x + sA[0][0].x * t.green[n];
            sR[0][0][n] = dcplx{0.0, ut};
            sR[0][1][n] = dcplx{0.0, -ut};
            sR[0][2][n] = dcplx{uz, 0.0};
            sP[0][n] = dcplx{0.0, 0.0};
        }
    }
    __syncthreads();

    // ---- output u (r, theta, z); vorticity from the stored components -------
    // omega is computed from (u_r, u_theta, u_z) as stored, so it equals what
    // the standalone vorticity kernel gives for the same state (bitwise
    // resumable runs).
    const bool mirror = (mi == 0 && kabs > 0);  // m = 0: -k is the conjugate of +k
    if (n < N) {
        for (int s = 0; s < nsig; ++s) {
            const int k = s == 0 ? kabs : -kabs;
            const dcplx up = sR[s][0][n], um = sR[s][1][n], uz = sR[s][2][n];
            const dcplx ur = 0.5 * (up + um), ut = 0.5 * dcplx{(up - um).y, -(up - um).x};
            const dcplx uo[3] = {ur, ut, uz};
            const size_t off = ((size_t)mi * nk + (k + K - 1)) * N + n;
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
                const dcplx p = sP[s][n];
                store_c<double>(a.p_out, off, p);
                if (mirror) store_c<double>(a.p_out, offc, dcplx{p.x, -p.y});
            }
            sU[s][0][n] = ur + ix(ut);
            sU[s][1][n] = ur - ix(ut);
            sU[s][2][n] = uz;
        }
    }
    __syncthreads();
    if (a.w_out && n < N) {
        for (int s = 0; s < nsig; ++s) {
            const int k = s == 0 ? kabs : -kabs;
            dcplx wp, wm, wz;
            vort_row(t, N, n, m, a.alpha * k, sU[s][0], sU[s][1], sU[s][2], wp, wm, wz);
            const dcplx wo[3] = {0.5 * (wp + wm), 0.5 * dcplx{(wp - wm).y, -(wp - wm).x}, wz};
            const size_t off = ((size_t)mi * nk + (k + K - 1)) * N + n;
            const size_t offc = ((size_t)mi * nk + (K - 1 - kabs)) * N + n;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                store_c<TNL>(a.w_out, c * S + off, wo[c]);
                if (mirror) store_c<TNL>(a.w_out, c * S + offc, dcplx{wo[c].x, -wo[c].y});
            }
        }
    }
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

hipError_t launch_solve(const SolveArgs& a, int precision, hipStream_t s) {
    const dim3 grid(a.M * a.K), block(64);
    if (precision == OPF_MIXED)
        hipLaunchKernelGGL(k_solve<float>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(k_solve<double>, grid, block, 0, s, a);
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
