// Dealiased pseudospectral nonlinear term u x omega on MI355X (CDNA4).
//
// Section 2 of the paper: the Fourier sums of Eq. (1) are evaluated on a
// 3K x 3M grid (3/2 rule), products are formed in physical space and
// transformed back (Section 2.2: nonlinear terms are evaluated
// pseudospectrally); the transform is two FFT stages with a data reordering
// between them (Section 2.2).  Here the two stages are three kernels:
//
//   k_zinv  : per (field, m, 8 radial nodes): 2K-1 axial coefficients ->
//             3K points (inverse c2c, zero padded), written z-contiguous to
//             H[field][n][m][z].
//   k_theta_lp : per (n, 4 axial points): the 6 fields' M azimuthal
//             coefficients are packed two real fields per complex line,
//             inverse FFT over 3M points, u x omega at every point, forward
//             FFT of (N_r + i N_t) and (N_z + i 0), unpacked and scaled by
//             1/(9KM) into G[comp][n][m][z].  Physical fields never leave LDS.
//   k_zfwd  : per (comp, m, 8 radial nodes): forward c2c over 3K points,
//             |k| < K kept, written to the spectral layout.
//
// Each length is split L = RA RB: a radix-RA DFT in registers per lane, a
// reordering through LDS with the twiddles W_L^{j r} (host-built table staged
// in LDS), then a radix-RB DFT; the roots inside each radix are compile-time
// constants.
#include "opf_internal.h"

namespace opf {

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // a * conj(b)
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }

// In-register DFT of length R; sign = -1 forward, +1 inverse.
template <typename T, int R>
__device__ __forceinline__ void dft(cpx<T>* v, int sign) {
    if constexpr (R == 2) {
        cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const T h = T(0.86602540378443864676);  // sin(2 pi / 3)
        cpx<T> a = v[0], b = v[1], c = v[2];
        cpx<T> s = cadd(b, c), d = csub(b, c);
        cpx<T> t = {a.x - T(0.5) * s.x, a.y - T(0.5) * s.y};
        // i * sign * h * d
        cpx<T> e = {-T(sign) * h * d.y, T(sign) * h * d.x};
        v[0] = cadd(a, s);
        v[1] = cadd(t, e);
        v[2] = csub(t, e);
    } else {  // R == 4
        cpx<T> a = v[0], b = v[1], c = v[2], d = v[3];
        cpx<T> t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), bd = csub(b, d);
        cpx<T> t3 = {-T(sign) * bd.y, T(sign) * bd.x};  // i * sign * (b - d)
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
}

template <typename TO, typename TI>
__device__ __forceinline__ cpx<TO> cvt(cpx<TI> a) { return {TO(a.x), TO(a.y)}; }

// Small DFT of length R in registers, R in {2,3,4,6,8,9,12,16}.
// - Composite R = R1 R2 (R1 in {3,4}) by one Cooley-Tukey split: R2 DFTs of
//   length R1 on stride-R2 subsets, twiddles W_R^{n2 k1}, R1 DFTs of length
//   R2; output index k1 + R1 k2.  The twiddles W_R^e are compile-time
//   constants.
// - With PF set, R = 6 and 12 = R1 3 (R1 in {2, 4}, prime to 3) take the
//   prime-factor (Good-Thomas) split instead, which needs no twiddles: input
//   n = (3 n1 + R1 n2) mod R, DFTs of length R1 over n1, then of length 3
//   over n2; output k is the residue pair (k mod R1, k mod 3) = (k1, k2)
//   rebuilt by the Chinese remainder theorem.  It saves the 6 twiddle
//   products of a 12-point DFT (two of them by 0 and +-1, which the compiler
//   may not fold), about a tenth of the theta stage's VALU instructions.
template <int R> struct Split1 { static constexpr int R1 = (R == 6 || R == 9) ? 3 : 4; };
constexpr int crt_coef(int a, int m) {  // a (a^-1 mod m): 1 mod m, 0 mod a
    int i = 0;
    while ((a * i) % m != 1 % m) ++i;
    return a * i;
}

// cos and sin of 2 pi e / R, evaluated by the compiler: the angle is reduced
// exactly to y = 2 pi e / R - o pi / 2 with |y| <= pi / 4 (o the nearest
// quarter turn), and cos y, sin y are summed from their Taylor series to
// well below double rounding.
constexpr double kPi = 3.14159265358979323846;
constexpr double taylor_cos(double y) {
    double t = 1.0, s = 1.0;
    for (int i = 1; i <= 12; ++i) { t *= -y * y / ((2 * i - 1) * (2 * i)); s += t; }
    return s;
}
constexpr double taylor_sin(double y) {
    double t = y, s = y;
    for (int i = 1; i <= 12; ++i) { t *= -y * y / ((2 * i) * (2 * i + 1)); s += t; }
    return s;
}
template <int R>
struct UnitRoots {
    double c[R], s[R];  // cos, sin of 2 pi e / R
    constexpr UnitRoots() : c(), s() {
        for (int e = 0; e < R; ++e) {
            const int o = (8 * e + R) / (2 * R);  // nearest multiple of R / 4 to e, in quarters
            const double y = (kPi / 2) * double(4 * e - o * R) / double(R);
            const double cy = taylor_cos(y), sy = taylor_sin(y);
            switch (o % 4) {
                case 0: c[e] = cy; s[e] = sy; break;
                case 1: c[e] = -sy; s[e] = cy; break;
                case 2: c[e] = -cy; s[e] = -sy; break;
                default: c[e] = sy; s[e] = -cy; break;
            }
        }
    }
};
template <int R> struct RootTable { static constexpr UnitRoots<R> v{}; };

// W_R^e = e^{-2 pi i e / R}
template <typename T, int R>
__device__ __forceinline__ cpx<T> unit_root(int e) {
    return {T(RootTable<R>::v.c[e]), T(-RootTable<R>::v.s[e])};
}

template <typename T, int R, bool PF = false>
__device__ __forceinline__ void dftn(cpx<T>* v, int sign) {
    if constexpr (R <= 4) {
        dft<T, R>(v, sign);
    } else if constexpr (PF && (R == 6 || R == 12)) {
        constexpr int R1 = R / 3, C1 = crt_coef(3, R1), C2 = crt_coef(R1, 3);
        cpx<T> y[3][R1];
#pragma unroll
        for (int n2 = 0; n2 < 3; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = v[(3 * n1 + R1 * n2) % R];
            dft<T, R1>(y[n2], sign);
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            cpx<T> z[3] = {y[0][k1], y[1][k1], y[2][k1]};
            dft<T, 3>(z, sign);
#pragma unroll
            for (int k2 = 0; k2 < 3; ++k2) v[(C1 * k1 + C2 * k2) % R] = z[k2];
        }
    } else {
        constexpr int R1 = Split1<R>::R1, R2 = R / R1;
        cpx<T> y[R2][R1];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = v[R2 * n1 + n2];
            dft<T, R1>(y[n2], sign);
        }
#pragma unroll
        for (int n2 = 1; n2 < R2; ++n2)
#pragma unroll
            for (int k1 = 1; k1 < R1; ++k1) {
                const cpx<T> w = unit_root<T, R>((n2 * k1) % R);
                y[n2][k1] = sign < 0 ? cmul(y[n2][k1], w) : cmulc(y[n2][k1], w);
            }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            cpx<T> z[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) z[n2] = y[n2][k1];
            dft<T, R2>(z, sign);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = z[k2];
        }
    }
}

// Two-pass factorisation L = RA * RB of every supported transform length.
// Pass A (radix RA): thread j < RB takes x[j + r RB], r < RA, and produces
// y[j RA + r].  Pass B (radix RB): thread j < RA takes y[j + r RA], r < RB,
// multiplies by W_L^{j r} and produces X[j + r RA].
template <int L> struct TwoPass;
template <> struct TwoPass<6> { static constexpr int RA = 2, RB = 3; };
template <> struct TwoPass<9> { static constexpr int RA = 3, RB = 3; };
template <> struct TwoPass<12> { static constexpr int RA = 3, RB = 4; };
template <> struct TwoPass<18> { static constexpr int RA = 3, RB = 6; };
template <> struct TwoPass<24> { static constexpr int RA = 4, RB = 6; };
template <> struct TwoPass<36> { static constexpr int RA = 6, RB = 6; };
template <> struct TwoPass<48> { static constexpr int RA = 6, RB = 8; };
template <> struct TwoPass<54> { static constexpr int RA = 6, RB = 9; };
template <> struct TwoPass<72> { static constexpr int RA = 8, RB = 9; };
template <> struct TwoPass<96> { static constexpr int RA = 8, RB = 12; };
template <> struct TwoPass<108> { static constexpr int RA = 9, RB = 12; };
template <> struct TwoPass<144> { static constexpr int RA = 12, RB = 12; };
template <> struct TwoPass<192> { static constexpr int RA = 12, RB = 16; };
template <int L>
__host__ __device__ constexpr int radix_max() {
    return TwoPass<L>::RA > TwoPass<L>::RB ? TwoPass<L>::RA : TwoPass<L>::RB;
}

// Segment strides of the z transforms' skewed LDS layout (the layout is
// described at k_theta_lp): LSI for k_zinv, LSF for k_zfwd, chosen the same
// way for these kernels' lane orders.
template <int L> struct ZLayout;
template <> struct ZLayout<6> { static constexpr int LSI = 10, LSF = 19; };
template <> struct ZLayout<9> { static constexpr int LSI = 13, LSF = 19; };
template <> struct ZLayout<12> { static constexpr int LSI = 18, LSF = 18; };
template <> struct ZLayout<18> { static constexpr int LSI = 26, LSF = 38; };
template <> struct ZLayout<24> { static constexpr int LSI = 30, LSF = 38; };
template <> struct ZLayout<36> { static constexpr int LSI = 42, LSF = 54; };
template <> struct ZLayout<48> { static constexpr int LSI = 70, LSF = 58; };
template <> struct ZLayout<54> { static constexpr int LSI = 70, LSF = 73; };
template <> struct ZLayout<72> { static constexpr int LSI = 81, LSF = 89; };
template <> struct ZLayout<96> { static constexpr int LSI = 110, LSF = 110; };
template <> struct ZLayout<108> { static constexpr int LSI = 126, LSF = 122; };
template <> struct ZLayout<144> { static constexpr int LSI = 158, LSF = 158; };
template <> struct ZLayout<192> { static constexpr int LSI = 210, LSF = 210; };
// LDS bytes of one z-transform workgroup
template <typename T, int L, bool INV, int ZT>
constexpr size_t z_lds() {
    return (size_t)(radix_max<L>() * radix_max<L>() + ZT * (INV ? ZLayout<L>::LSI : ZLayout<L>::LSF)) * sizeof(cpx<T>);
}

// Threads of a z-transform workgroup: 128, or 256 when ZT radial lines of
// the longer radix pass need more (ZT max(RA, RB) <= 256).
template <int L, int ZT>
constexpr int z_threads() { return ZT * radix_max<L>() <= 128 ? 128 : 256; }

// ---------------------------------------------------------------------------
// k_zinv: spectral [M][nk][N] -> H[f][n][m][z], z = 0..3K-1 (inverse, zero
// padded).  Workgroup: field f, azimuthal index m, ZT radial nodes.
template <typename TS, typename T, int L, int ZT>
__device__ __forceinline__ void k_zinv_body(const NLArgs& a) {
    constexpr int RA = TwoPass<L>::RA, RB = TwoPass<L>::RB, LS = ZLayout<L>::LSI, RM = radix_max<L>();
    static_assert(LS >= L + RM, "segment too short for the skewed layout");
    constexpr int NT2 = z_threads<L, ZT>();
    static_assert(ZT * RM <= NT2, "a pass must fit the workgroup");
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* tw2 = reinterpret_cast<cpx<T>*>(smem_raw);  // [RM][RM]: W_L^{j r} at r RM + j
    // prime-factor split in FP32 only: measured 6% faster there, 7% slower in
    // FP64 (a bandwidth-bound kernel, which the twiddle products do not limit)
    constexpr bool ZPF = sizeof(T) == 4;
    cpx<T>* buf = tw2 + RM * RM;                         // [ZT][LS]
    constexpr int K = L / 3, nk = 2 * K - 1;  // the z line is the 3/2-padded length 3K
    const int N = a.N, M = a.M;
    const int ntile = (N + ZT - 1) / ZT;
    const int tile = blockIdx.x % ntile;
    const int m = (blockIdx.x / ntile) % M;
    const int f = blockIdx.x / (ntile * M);
    const int n0 = tile * ZT;
    const int tid = threadIdx.x;
    const cpx<T>* twg = reinterpret_cast<const cpx<T>*>(a.twz);  // W_L^t, t < L
    for (int t = tid; t < RM * RM; t += NT2) tw2[t] = twg[((t % RM) * (t / RM)) % L];
    const cpx<TS>* src = reinterpret_cast<const cpx<TS>*>(a.in[f]) + (size_t)m * nk * N;
    // pass A: thread (j, nn), radial node fastest (coalesced rows of the spectral layout)
    const int ja = tid / ZT, na = tid % ZT;
    cpx<T> v[RA];
    if (ja < RB) {
        const int n = min(n0 + na, N - 1);
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const int bin = ja + r * RB;
            int kk = -1;
            if (bin < K) kk = bin + K - 1;
            else if (bin > L - K) kk = bin - L + K - 1;
            v[r] = kk >= 0 ? cvt<T>(src[(size_t)kk * N + n]) : cpx<T>{T(0), T(0)};
        }
        dftn<T, RA, ZPF>(v, +1);
#pragma unroll
        for (int r = 0; r < RA; ++r) buf[na * LS + r * (RB + 1) + ja] = v[r];
    }
    __syncthreads();  // pass A results and tw2
    // pass B: thread (nn, j), z fastest (coalesced z lines of H)
    const int nb = tid / RA, jb = tid % RA;
    if (nb < ZT && n0 + nb < N) {
        cpx<T> u[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const cpx<T> x = buf[nb * LS + jb * (RB + 1) + r];  // output jb of pass-A lane r
            u[r] = r == 0 ? x : cmulc(x, tw2[r * RM + jb]);
        }
        dftn<T, RB, ZPF>(u, +1);
        cpx<T>* dst = reinterpret_cast<cpx<T>*>(a.H) + ((size_t)f * N * M + (size_t)(n0 + nb) * M + m) * L;
#pragma unroll
        for (int r = 0; r < RB; ++r) dst[jb + r * RA] = u[r];
    }
}

template <typename TS, typename T, int L, int ZT>
__global__ __launch_bounds__((z_threads<L, ZT>())) void k_zinv(NLArgs a) { k_zinv_body<TS, T, L, ZT>(a); }
template <typename TS, typename T, int L, int ZT>
__global__ __launch_bounds__((z_threads<L, ZT>())) void k_zinv_b(const NLArgs* __restrict__ aa) {
    k_zinv_body<TS, T, L, ZT>(aa[blockIdx.y]);  // record read in place, not copied to scratch
}

// Coriolis force -2 Omega x u added to (nr, nt, nz) at theta point t of the
// dealiased line: angle 2 pi t / 3M (a transverse axis needs mp = 1), with
// w = exp(-2 pi i t / 3M) giving its cosine and sine.
template <typename T>
__device__ __forceinline__ void add_coriolis(const NLArgs& a, cpx<T> w, T ur, T ut, T uz, T& nr, T& nt, T& nz) {
    const T c = w.x, s = -w.y;
    const T ox = T(a.rot[0]), oy = T(a.rot[1]), oz = T(a.rot[2]);
    const T o_r = ox * c + oy * s, o_t = oy * c - ox * s;
    nr -= T(2) * (o_t * uz - oz * ut);
    nt -= T(2) * (oz * ur - o_r * uz);
    nz -= T(2) * (o_r * ut - o_t * ur);
}

// ---------------------------------------------------------------------------
// k_theta_lp: per (n, TZ axial points; TZ = 2, 4 or 8 with TZ max(RA, RB)
// <= 64), the three packed lines spread
// over the three waves of a 192-thread workgroup (wave p holds line p).  A
// thread keeps one line's RA or RB values, not all three (an FP64 thread
// holding all three needs 208 VGPRs), and the product reads the three lines
// from LDS.  Workgroups are ordered so that the tiles sharing a 128-byte
// line of H and G (2 in FP64, 4 in FP32) run on the same XCD, consecutive
// block indices being dispatched round-robin over the 8 XCDs.
//
// LDS layout.  Each wave owns TZ segments of LS slots (one per axial point).
// Between the two radix passes of a transform, the r-th output of first-pass
// lane j sits at slot r (R2 + 1) + j, R2 the number of first-pass lanes of a
// line: the first pass stores at stride one across lanes and the second pass
// loads at stride R2 + 1.  Theta points (for the product) and wavenumber
// bins (for the unpacking) are kept in natural order.  LS >= L + max(RA, RB)
// is the padding that, among the 17 values from there, spreads the kernel's
// 16-byte accesses over the most LDS banks (64 four-byte banks, 16
// consecutive lanes), counted access by access.  The twiddles between the
// passes come from tw2[r RM + j] = W_L^{j r}, RM = max(RA, RB), read at
// stride one; the roots inside each radix are compile-time constants.
constexpr int TZC = 4;  // axial points per workgroup of the CFL kernel
constexpr int NT3 = 192;

template <int L> struct ThetaLayout;
template <> struct ThetaLayout<6> { static constexpr int LS = 13; };
template <> struct ThetaLayout<9> { static constexpr int LS = 19; };
template <> struct ThetaLayout<12> { static constexpr int LS = 20; };
template <> struct ThetaLayout<18> { static constexpr int LS = 28; };
template <> struct ThetaLayout<24> { static constexpr int LS = 44; };
template <> struct ThetaLayout<36> { static constexpr int LS = 54; };
template <> struct ThetaLayout<48> { static constexpr int LS = 70; };
template <> struct ThetaLayout<54> { static constexpr int LS = 70; };
template <> struct ThetaLayout<72> { static constexpr int LS = 88; };
template <> struct ThetaLayout<96> { static constexpr int LS = 120; };
template <> struct ThetaLayout<108> { static constexpr int LS = 121; };
template <> struct ThetaLayout<144> { static constexpr int LS = 156; };
template <> struct ThetaLayout<192> { static constexpr int LS = 220; };

// LDS bytes of one k_theta_lp workgroup
template <typename T, int L, int TZ>
constexpr size_t theta_lp_lds() {
    constexpr int tw = TwoPass<L>::RA == TwoPass<L>::RB ? 0 : radix_max<L>() * radix_max<L>();  // RA = RB: twiddles in registers
    return (size_t)(tw + 3 * TZ * ThetaLayout<L>::LS) * sizeof(cpx<T>);
}

// Blocks g*8G + x + 8y (x < 8, y < G) take tiles g*8G + G x + y, so the G
// tiles of one 128-byte line run on one XCD; a last partial group keeps the
// identity order.
template <int G>
__device__ __forceinline__ int xcd_group_tile(int b, int total) {
    const int g = b / (8 * G), w = b % (8 * G);
    if ((g + 1) * 8 * G > total) return b;
    return g * 8 * G + G * (w % 8) + w / 8;
}

template <typename T, int L, bool ROT, int TZ>
__device__ __forceinline__ void k_theta_lp_body(const NLArgs& a) {
    constexpr int RA = TwoPass<L>::RA, RB = TwoPass<L>::RB, LS = ThetaLayout<L>::LS, RM = radix_max<L>();
    constexpr int XG = 128 / (TZ * (int)sizeof(cpx<T>)) > 0 ? 128 / (TZ * (int)sizeof(cpx<T>)) : 1;  // tiles per 128-byte line of H and G
    static_assert(RA * TZ <= 64 && RB * TZ <= 64, "a line pass must fit one wave");
    static_assert(LS >= L + RM, "segment too short for the skewed layout");
    // RA = RB: a lane's twiddles W_L^{j r} are the same in the inverse pass B
    // and the forward pass B' (j = lane % RA in both), so each lane keeps its
    // RA - 1 values in registers and no table is staged in LDS
    constexpr bool TWREG = RA == RB;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* tw2 = reinterpret_cast<cpx<T>*>(smem_raw);  // [RM][RM]: W_L^{j r} at r RM + j (RA != RB)
    cpx<T>* buf = TWREG ? tw2 : tw2 + RM * RM;           // [3][TZ][LS]
    constexpr int M = L / 3;  // the theta line is the 3/2-padded length 3M
    const int N = a.N, L3K = 3 * a.K;
    const int nzt = (L3K + TZ - 1) / TZ;
    const int tile = xcd_group_tile<XG>(blockIdx.x, N * nzt);
    const int n = tile / nzt;
    const int z0 = (tile % nzt) * TZ;
    const int tid = threadIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const cpx<T>* twg = reinterpret_cast<const cpx<T>*>(a.twt);  // W_L^t, t < L
    if constexpr (!TWREG)
        for (int t = tid; t < RM * RM; t += NT3) tw2[t] = twg[((t % RM) * (t / RM)) % L];
    const cpx<T>* H = reinterpret_cast<const cpx<T>*>(a.H);
    const size_t fstride = (size_t)N * M * L3K;
    const size_t nbase = (size_t)n * M * L3K;
    cpx<T>* lb = buf + p * TZ * LS;  // this wave's line
    // inverse pass A: lane (j, zz), z fastest; bins j + r RB of line p = fields (2p, 2p+1)
    const int ja = lane / TZ, za = lane % TZ;
    const int zc = min(z0 + za, L3K - 1);
    cpx<T> v[RA];
    if (ja < RB) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const int bin = ja + r * RB;
            int mm = -1;
            bool neg = false;
            if (bin < M) mm = bin;
            else if (bin > L - M) { mm = L - bin; neg = true; }
            cpx<T> val = {T(0), T(0)};
            if (mm >= 0) {
                const size_t off = nbase + (size_t)mm * L3K + zc;
                const cpx<T> A = H[(2 * p) * fstride + off];
                const cpx<T> B = H[(2 * p + 1) * fstride + off];
                // Z = A + i B on m >= 0; conj(A) + i conj(B) on bins L - m
                val = neg ? cpx<T>{A.x + B.y, B.x - A.y} : cpx<T>{A.x - B.y, A.y + B.x};
            }
            v[r] = val;
        }
        dftn<T, RA, true>(v, +1);
#pragma unroll
        for (int r = 0; r < RA; ++r) lb[za * LS + r * (RB + 1) + ja] = v[r];
    }
    // inverse pass B: lane (zz, j); output r of pass-A lane r', then theta
    // points j + r RA in natural order
    const int zb = lane / RA, jb = lane % RA;
    cpx<T> twr[RA];  // W_L^{jb r} (TWREG)
    if constexpr (TWREG) {
#pragma unroll
        for (int r = 1; r < RA; ++r) twr[r] = twg[(jb * r) % L];
        __builtin_amdgcn_wave_barrier();  // pass A results: this wave's own line
    } else {
        __syncthreads();  // pass A results and tw2
    }
    const bool actB = zb < TZ;
    cpx<T> u[RB];
    if (actB) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const cpx<T> x = lb[zb * LS + jb * (RB + 1) + r];
            u[r] = r == 0 ? x : cmulc(x, TWREG ? twr[r] : tw2[r * RM + jb]);
        }
        dftn<T, RB, true>(u, +1);
    }
    __builtin_amdgcn_wave_barrier();  // the line is this wave's own: LDS accesses stay in order
    if (actB) {
#pragma unroll
        for (int r = 0; r < RB; ++r) lb[zb * LS + jb + r * RA] = u[r];
    }
    __syncthreads();
    // u x omega from the three lines; waves 0, 1 form (N_r + i N_t), (N_z + i 0)
    // and run forward pass A' (radix RB on the same points)
    const bool out = p < 2;
    if (out && actB) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int pt = jb + r * RA;
            const cpx<T> l0 = buf[zb * LS + pt], l1 = buf[(TZ + zb) * LS + pt], l2 = buf[(2 * TZ + zb) * LS + pt];
            const T ur = l0.x, ut = l0.y, uz = l1.x, wr = l1.y, wt = l2.x, wz = l2.y;
            T nr = ut * wz - uz * wt, nt = uz * wr - ur * wz, nz = ur * wt - ut * wr;
            // W_L^{jb + r RA} = W_L^{jb} W_RB^{r}
            if constexpr (ROT) add_coriolis<T>(a, cmul(TWREG ? twr[1] : tw2[RM + jb], unit_root<T, RB>(r)), ur, ut, uz, nr, nt, nz);
            u[r] = p == 0 ? cpx<T>{nr, nt} : cpx<T>{nz, T(0)};
        }
        dftn<T, RB, true>(u, -1);
    }
    __syncthreads();  // every line has been read
    if (out && actB) {
#pragma unroll
        for (int r = 0; r < RB; ++r) lb[zb * LS + r * (RA + 1) + jb] = u[r];
    }
    __builtin_amdgcn_wave_barrier();  // pass B' reads this wave's own line
    // forward pass B' (radix RA): lane (zz, j), j < RB, takes output j of
    // pass-A' lanes r = 0..RA-1; results are bins j + r RB
    const int zc2 = lane / RB, jc = lane % RB;
    const bool actC = out && zc2 < TZ;
    cpx<T> x2[RA];
    if (actC) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const cpx<T> x = lb[zc2 * LS + jc * (RA + 1) + r];
            x2[r] = r == 0 ? x : cmul(x, TWREG ? twr[r] : tw2[r * RM + jc]);
        }
        dftn<T, RA, true>(x2, -1);
    }
    __builtin_amdgcn_wave_barrier();
    if (actC) {
#pragma unroll
        for (int r = 0; r < RA; ++r) lb[zc2 * LS + jc + r * RB] = x2[r];
    }
    __syncthreads();
    // unpack the two output lines and store G (scaled by 1/(9KM))
    cpx<T>* G = reinterpret_cast<cpx<T>*>(a.G);
    const T h = T(0.5) * T(a.scale);
    for (int t = tid; t < 2 * M * TZ; t += NT3) {
        const int q = t / (M * TZ), rem = t % (M * TZ);
        const int mm = rem / TZ, zz = rem % TZ, z = z0 + zz;
        if (z >= L3K) continue;
        const int mc = mm == 0 ? 0 : L - mm;
        const cpx<T>* line = buf + (q * TZ + zz) * LS;
        const cpx<T> Z = line[mm], Y = line[mc];
        const size_t off = nbase + (size_t)mm * L3K + z;
        if (q == 0) {  // A = (Z + conj Y)/2 -> N_r, B = (Z - conj Y)/(2i) -> N_t
            G[off] = {h * (Z.x + Y.x), h * (Z.y - Y.y)};
            G[fstride + off] = {h * (Z.y + Y.y), h * (Y.x - Z.x)};
        } else {
            G[2 * fstride + off] = {h * (Z.x + Y.x), h * (Z.y - Y.y)};
        }
    }
}

template <typename T, int L, bool ROT, int TZ>
__global__ __launch_bounds__(NT3) void k_theta_lp(NLArgs a) { k_theta_lp_body<T, L, ROT, TZ>(a); }
template <typename T, int L, int TZ>
__global__ __launch_bounds__(NT3) void k_theta_lp_b(const NLArgs* __restrict__ aa) {
    k_theta_lp_body<T, L, false, TZ>(aa[blockIdx.y]);  // ensemble members carry no forcing
}

// ---------------------------------------------------------------------------
// k_cfl: per (n, TZ axial points) the velocity lines (u_r + i u_theta) and
// (u_z + i omega_r) are transformed to theta points as in k_theta_lp (wave p
// holds line p), then out[block] = max over the tile's points of
// |u_r| wr[n] + |u_theta| wt[n] + |u_z| wz (the local CFL rate).
template <typename T, int L>
__global__ __launch_bounds__(128) void k_cfl(NLArgs a, const double* __restrict__ wr, const double* __restrict__ wt,
                                             double wz, double* __restrict__ out) {
    constexpr int RA = TwoPass<L>::RA, RB = TwoPass<L>::RB, LS = L + 1;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);  // [L]
    cpx<T>* buf = tw + L;                                // [2][TZC][LS]
    constexpr int M = L / 3;  // the theta line is the 3/2-padded length 3M
    const int N = a.N, L3K = 3 * a.K;
    const int nzt = (L3K + TZC - 1) / TZC;
    const int n = blockIdx.x / nzt;
    const int z0 = (blockIdx.x % nzt) * TZC;
    const int tid = threadIdx.x;
    const int p = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const cpx<T>* twg = reinterpret_cast<const cpx<T>*>(a.twt);
    for (int t = tid; t < L; t += 128) tw[t] = twg[t];
    const cpx<T>* H = reinterpret_cast<const cpx<T>*>(a.H);
    const size_t fstride = (size_t)N * M * L3K;
    const size_t nbase = (size_t)n * M * L3K;
    cpx<T>* lb = buf + p * TZC * LS;
    const int ja = lane / TZC, za = lane % TZC;
    const int zc = min(z0 + za, L3K - 1);
    cpx<T> v[RA];
    if (ja < RB) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const int bin = ja + r * RB;
            int mm = -1;
            bool neg = false;
            if (bin < M) mm = bin;
            else if (bin > L - M) { mm = L - bin; neg = true; }
            cpx<T> val = {T(0), T(0)};
            if (mm >= 0) {
                const size_t off = nbase + (size_t)mm * L3K + zc;
                const cpx<T> A = H[(2 * p) * fstride + off];
                const cpx<T> B = H[(2 * p + 1) * fstride + off];
                val = neg ? cpx<T>{A.x + B.y, B.x - A.y} : cpx<T>{A.x - B.y, A.y + B.x};
            }
            v[r] = val;
        }
    }
    __syncthreads();  // twiddles
    if (ja < RB) {
        dftn<T, RA, true>(v, +1);
#pragma unroll
        for (int r = 0; r < RA; ++r) lb[za * LS + ja * RA + r] = v[r];
    }
    __syncthreads();
    const int zb = lane / RA, jb = lane % RA;
    const bool actB = zb < TZC;
    cpx<T> u[RB];
    if (actB) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const cpx<T> x = lb[zb * LS + jb + r * RA];
            u[r] = r == 0 ? x : cmulc(x, tw[jb * r]);
        }
        dftn<T, RB, true>(u, +1);
    }
    __syncthreads();
    if (actB) {
#pragma unroll
        for (int r = 0; r < RB; ++r) lb[zb * LS + jb + r * RA] = u[r];
    }
    __syncthreads();
    if (p == 0) {
        double mx = 0.0;
        if (actB) {
            const double a1 = wr[n], a2 = wt[n];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int pt = jb + r * RA;
                const cpx<T> l0 = buf[zb * LS + pt], l1 = buf[(TZC + zb) * LS + pt];
                mx = fmax(mx, fabs((double)l0.x) * a1 + fabs((double)l0.y) * a2 + fabs((double)l1.x) * wz);
            }
        }
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) out[blockIdx.x] = mx;
    }
}

#define OPF_FOR_LENGTHS_CFL(X) X(6) X(9) X(12) X(18) X(24) X(36) X(48) X(54) X(72) X(96) X(108) X(144) X(192)
template <typename T>
static hipError_t launch_cfl_typed(const NLArgs& a, const double* wr, const double* wt, double wz, double* out,
                                   hipStream_t s) {
    const int L3M = 3 * a.M;
    const dim3 g(a.N * ((3 * a.K + TZC - 1) / TZC));
    const size_t lds = (size_t)(L3M + 2 * TZC * (L3M + 1)) * sizeof(cpx<T>);
    switch (L3M) {
#define OPF_CASE(V)                                                                       \
    case V:                                                                               \
        hipLaunchKernelGGL((k_cfl<T, V>), g, dim3(128), lds, s, a, wr, wt, wz, out);      \
        break;
        OPF_FOR_LENGTHS_CFL(OPF_CASE)
#undef OPF_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_zfwd: G[f][n][m][z] -> spectral [M][nk][N] (forward), |k| < K kept.
template <typename TS, typename T, int L, int ZT>
__device__ __forceinline__ void k_zfwd_body(const NLArgs& a) {
    constexpr int RA = TwoPass<L>::RA, RB = TwoPass<L>::RB, LS = ZLayout<L>::LSF, RM = radix_max<L>();
    static_assert(LS >= L + RM, "segment too short for the skewed layout");
    constexpr int NT2 = z_threads<L, ZT>();
    static_assert(ZT * RM <= NT2, "a pass must fit the workgroup");
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* tw2 = reinterpret_cast<cpx<T>*>(smem_raw);  // [RM][RM]: W_L^{j r} at r RM + j
    cpx<T>* buf = tw2 + RM * RM;                         // [ZT][LS]
    constexpr int K = L / 3, nk = 2 * K - 1;  // the z line is the 3/2-padded length 3K
    const int N = a.N, M = a.M;
    const int ntile = (N + ZT - 1) / ZT;
    const int tile = blockIdx.x % ntile;
    const int m = (blockIdx.x / ntile) % M;
    const int f = blockIdx.x / (ntile * M);
    const int n0 = tile * ZT;
    const int tid = threadIdx.x;
    const cpx<T>* twg = reinterpret_cast<const cpx<T>*>(a.twz);  // W_L^t, t < L
    for (int t = tid; t < RM * RM; t += NT2) tw2[t] = twg[((t % RM) * (t / RM)) % L];
    const cpx<T>* src = reinterpret_cast<const cpx<T>*>(a.G) + (size_t)f * N * M * L;
    // pass A: thread (nn, j), z fastest
    const int na = tid / RB, ja = tid % RB;
    cpx<T> v[RA];
    if (na < ZT) {
        const int n = min(n0 + na, N - 1);
        const cpx<T>* line = src + ((size_t)n * M + m) * L;
#pragma unroll
        for (int r = 0; r < RA; ++r) v[r] = line[ja + r * RB];
        dftn<T, RA>(v, -1);
#pragma unroll
        for (int r = 0; r < RA; ++r) buf[na * LS + r * (RB + 1) + ja] = v[r];
    }
    __syncthreads();  // pass A results and tw2
    // pass B: thread (j, nn), radial node fastest (coalesced spectral rows)
    const int jb = tid / ZT, nb = tid % ZT;
    if (jb < RA && n0 + nb < N) {
        cpx<T> u[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const cpx<T> x = buf[nb * LS + jb * (RB + 1) + r];  // output jb of pass-A lane r
            u[r] = r == 0 ? x : cmul(x, tw2[r * RM + jb]);
        }
        dftn<T, RB>(u, -1);
        cpx<TS>* dst = reinterpret_cast<cpx<TS>*>(a.out[f]) + (size_t)m * nk * N + n0 + nb;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int bin = jb + r * RA;
            int kk = -1;
            if (bin < K) kk = bin + K - 1;
            else if (bin > L - K) kk = bin - L + K - 1;
            if (kk >= 0) dst[(size_t)kk * N] = cvt<TS>(u[r]);
        }
    }
}

template <typename TS, typename T, int L, int ZT>
__global__ __launch_bounds__((z_threads<L, ZT>())) void k_zfwd(NLArgs a) { k_zfwd_body<TS, T, L, ZT>(a); }
template <typename TS, typename T, int L, int ZT>
__global__ __launch_bounds__((z_threads<L, ZT>())) void k_zfwd_b(const NLArgs* __restrict__ aa) {
    k_zfwd_body<TS, T, L, ZT>(aa[blockIdx.y]);  // record read in place, not copied to scratch
}

// ---------------------------------------------------------------------------
// Host dispatch over the supported transform lengths 3K, 3M.
#define OPF_FOR_LENGTHS(X) X(6) X(9) X(12) X(18) X(24) X(36) X(48) X(54) X(72) X(96) X(108) X(144) X(192)

static bool length_ok(int L) {
#define OPF_CASE(V) if (L == V) return true;
    OPF_FOR_LENGTHS(OPF_CASE)
#undef OPF_CASE
    return false;
}

bool nonlinear_supported(int M, int K) { return length_ok(3 * M) && length_ok(3 * K); }

// Largest radix of the two-pass split of length L (0: unsupported length).
static int radix_of(int L) {
    switch (L) {
#define OPF_CASE(V) case V: return radix_max<V>();
        OPF_FOR_LENGTHS(OPF_CASE)
#undef OPF_CASE
        default: return 0;
    }
}

bool ztile_ok(int zt, int K) { return (zt == 4 || zt == 8 || zt == 16) && radix_of(3 * K) * zt <= 256; }
bool tz_ok(int tz, int M) { return (tz == 2 || tz == 4 || tz == 8) && radix_of(3 * M) * tz <= 64; }

template <typename TS, typename T, int L, int ZT>
static void launch_z(const NLArgs& a, const NLArgs* batch, int members, bool inv, hipStream_t s, const KernelTiming& kt) {
    const int ntile = (a.N + ZT - 1) / ZT;
    const bool b = batch != nullptr;
    if constexpr (ZT * radix_max<L>() <= 256) {
        constexpr int NT = z_threads<L, ZT>();
        if (inv) {
            const dim3 g(6 * a.M * ntile, b ? members : 1);
            if (b) hipLaunchKernelGGL((k_zinv_b<TS, T, L, ZT>), g, dim3(NT), (z_lds<T, L, true, ZT>()), s, batch);
            else launch_timed((k_zinv<TS, T, L, ZT>), g, dim3(NT), (z_lds<T, L, true, ZT>()), s, kt, a);
        } else {
            const dim3 g(3 * a.M * ntile, b ? members : 1);
            if (b) hipLaunchKernelGGL((k_zfwd_b<TS, T, L, ZT>), g, dim3(NT), (z_lds<T, L, false, ZT>()), s, batch);
            else launch_timed((k_zfwd<TS, T, L, ZT>), g, dim3(NT), (z_lds<T, L, false, ZT>()), s, kt, a);
        }
    }
}

template <typename T, int L, int TZ>
static void launch_theta(const NLArgs& a, const NLArgs* batch, int members, hipStream_t s, const KernelTiming& kt) {
    if constexpr (TZ * radix_max<L>() <= 64) {
        const dim3 g(a.N * ((3 * a.K + TZ - 1) / TZ), batch ? members : 1);
        if (batch) hipLaunchKernelGGL((k_theta_lp_b<T, L, TZ>), g, dim3(NT3), (theta_lp_lds<T, L, TZ>()), s, batch);
        else if (a.rotating) launch_timed((k_theta_lp<T, L, true, TZ>), g, dim3(NT3), (theta_lp_lds<T, L, TZ>()), s, kt, a);
        else launch_timed((k_theta_lp<T, L, false, TZ>), g, dim3(NT3), (theta_lp_lds<T, L, TZ>()), s, kt, a);
    }
}

template <typename TS, typename T>
static hipError_t launch_typed(const NLArgs& a, const NLArgs* batch, int members, int stage, hipStream_t s,
                               const KernelTiming& kt = KernelTiming{}) {
    const int L3K = 3 * a.K, L3M = 3 * a.M;
    if (stage == 1) {
        if (!tz_ok(a.tz, a.M)) return hipErrorInvalidValue;
        switch (L3M) {
#define OPF_CASE(V)                                                        \
    case V:                                                                \
        if (a.tz == 2) launch_theta<T, V, 2>(a, batch, members, s, kt);      \
        else if (a.tz == 4) launch_theta<T, V, 4>(a, batch, members, s, kt); \
        else launch_theta<T, V, 8>(a, batch, members, s, kt);                \
        break;
            OPF_FOR_LENGTHS(OPF_CASE)
#undef OPF_CASE
            default: return hipErrorInvalidValue;
        }
    } else {
        if (!ztile_ok(a.ztile, a.K)) return hipErrorInvalidValue;
        const bool inv = stage == 0;
        switch (L3K) {
#define OPF_CASE(V)                                                                \
    case V:                                                                        \
        if (a.ztile == 4) launch_z<TS, T, V, 4>(a, batch, members, inv, s, kt);      \
        else if (a.ztile == 8) launch_z<TS, T, V, 8>(a, batch, members, inv, s, kt); \
        else launch_z<TS, T, V, 16>(a, batch, members, inv, s, kt);                  \
        break;
            OPF_FOR_LENGTHS(OPF_CASE)
#undef OPF_CASE
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_nonlinear_batch(const NLArgs& proto, const NLArgs* dev_args, int members, int precision,
                                  int stage, hipStream_t s) {
    if (precision == OPF_MIXED) return launch_typed<float, float>(proto, dev_args, members, stage, s);
    return launch_typed<double, double>(proto, dev_args, members, stage, s);
}

hipError_t launch_nonlinear_stage(const NLArgs& a, int precision, int stage, hipStream_t s, const KernelTiming& kt) {
    if (precision == OPF_MIXED) return launch_typed<float, float>(a, nullptr, 1, stage, s, kt);
    return launch_typed<double, double>(a, nullptr, 1, stage, s, kt);
}

hipError_t launch_cfl(const NLArgs& a, int precision, const double* wr, const double* wt, double wz, double* out,
                      hipStream_t s) {
    if (!length_ok(3 * a.M)) return hipErrorInvalidValue;
    if (precision == OPF_MIXED) return launch_cfl_typed<float>(a, wr, wt, wz, out, s);
    return launch_cfl_typed<double>(a, wr, wt, wz, out, s);
}

hipError_t launch_nonlinear(const NLArgs& a, int precision, hipStream_t s) {
    for (int stage = 0; stage < 3; ++stage) {
        const hipError_t e = launch_nonlinear_stage(a, precision, stage, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace opf
