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
// imaginary part of one component of one mode) and walks the rows of the
// operator's substitution image (unit triangles of the diagonally scaled LU
// factors, see solve_image_doubles), brought into LDS by DMA.  About 52 KB
// of LDS and at most 168 VGPRs let three workgroups share a compute unit, so
// the 768 tiles of the 64 x 48 x 127-mode grid run in one round.  m = 0
// solves k >= 0 only and writes the conjugate into -k (Hermitian symmetry
// of a real field); mode (0,0) has u_r = 0, no pressure and the fixed-flux
// correction.
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

template <typename T>
__device__ __forceinline__ dcplx load_c(const void* base, size_t idx) {
    const T* p = reinterpret_cast<const T*>(base) + 2 * idx;
    return {double(p[0]), double(p[1])};
}
// A complex value as stored (two T), read now and widened where it is used.
template <typename T>
struct vec2 {
    T x, y;
};
template <typename T>
__device__ __forceinline__ vec2<T> load_v(const void* base, size_t idx) {
    const T* p = reinterpret_cast<const T*>(base) + 2 * idx;
    return {p[0], p[1]};
}
template <typename T>
__device__ __forceinline__ dcplx to_c(vec2<T> v) {
    return {double(v.x), double(v.y)};
}
template <typename T>
__device__ __forceinline__ void store_c(void* base, size_t idx, dcplx v) {
    T* p = reinterpret_cast<T*>(base) + 2 * idx;
    p[0] = T(v.x);
    p[1] = T(v.y);
}

// Vorticity of mode (m, kappa) at one radial node, the cylindrical curl
// (the rotational form of the nonlinear term, Section 2.2):
//   w_r = (i m / r) u_z - i kappa u_theta,  w_theta = i kappa u_r - u_z',
//   w_z = u_theta' + (u_theta - i m u_r) / r,
// from the node's values and the radial derivatives duz = u_z' (parity of
// m) and dut = u_theta' (parity of m +- 1).
__device__ __forceinline__ void curl_row(dcplx duz, dcplx dut, double rinv, int m, double kap, dcplx ur, dcplx ut,
                                         dcplx uz, dcplx& wr, dcplx& wt, dcplx& wz) {
    wr = (double(m) * rinv) * ix(uz) - kap * ix(ut);
    wt = kap * ix(ur) - duz;
    wz = dut + rinv * (ut - double(m) * ix(ur));
}

// Substitution on one real right-hand side held in LDS (element i at
// col[2 i]: the real or imaginary part of a complex radial line; rows past
// N are zero), with a factor image F in LDS (see solve_image_doubles); one
// lane per right-hand side.  Forward sweep with the unit lower Lh, right-
// looking: once y_i is known it updates the next four (eight from row NW on)
// entries, kept in registers, so one multiply-add per row lies on the
// dependency chain; backward sweep with the unit upper W likewise.
//
// The sweeps are bound by LDS latency: a row's factor record and right-hand-
// side entry are read DN rows ahead (DW for the wide rows past NW, whose
// records are twice as long), within the register budget of three
// workgroups per compute unit.  Rows go in pairs so that the two entries
// read and the two results written become one ds_read2 / ds_write2 each:
// three LDS instructions per row, which keeps about five rows in flight
// under the LDS counter's limit of 15.  Each pair's instructions stay in
// place (a scheduling barrier per pair): free scheduling would hoist the
// reads of many rows at once.
template <int NB, int NW>
__device__ __forceinline__ void lds_solve(const double* __restrict__ F, double* col) {
    constexpr int DN = 6, DW = 4, DB = 6;  // read-ahead in rows: narrow and wide forward rows, backward rows
    static_assert(NB % 2 == 0, "rows go in pairs");
    constexpr int FWD = solve_image_fwd(NB, NW);
    auto frow = [](int i) { return i < NW ? 4 * i : 4 * NW + 8 * (i - NW); };
    auto brow = [](int i) { return FWD + 4 * (i - 1); };
    // row r is requested just before row issue(r) is computed (r <= 7: before the sweep)
    auto fissue = [](int r) { return r - (r < NW ? DN : DW); };
    double2 Lr[NB][4];
    double nb[NB];  // col[2 (r + 8)] for row r
    auto fload = [&](int r) {
        const double2* f = reinterpret_cast<const double2*>(F + frow(r));
#pragma unroll
        for (int j = 0; j < (r < NW ? 2 : 4); ++j) Lr[r][j] = f[j];
        nb[r] = r + 8 < NB ? col[2 * (r + 8)] : 0.0;
    };
#pragma unroll
    for (int r = 0; r < NB; ++r)
        if (fissue(r) < 0) fload(r);
    double b0 = col[0], b1 = col[2], b2 = col[4], b3 = col[6];
    double b4 = col[8], b5 = col[10], b6 = col[12], b7 = col[14];
#pragma unroll
    for (int i = 0; i < NB; i += 2) {
#pragma unroll
        for (int r = i + 1; r < NB && r <= i + 1 + DN; ++r)
            if (fissue(r) == i || fissue(r) == i + 1) fload(r);
        __builtin_amdgcn_sched_barrier(0);
        double y[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = i + h;
            y[h] = b0;
            b0 = b1 - Lr[r][0].x * y[h];
            b1 = b2 - Lr[r][0].y * y[h];
            b2 = b3 - Lr[r][1].x * y[h];
            b3 = b4 - Lr[r][1].y * y[h];
            if (r < NW) {
                b4 = b5;
                b5 = b6;
                b6 = b7;
                b7 = nb[r];
            } else {
                b4 = b5 - Lr[r][2].x * y[h];
                b5 = b6 - Lr[r][2].y * y[h];
                b6 = b7 - Lr[r][3].x * y[h];
                b7 = nb[r] - Lr[r][3].y * y[h];
            }
        }
        col[2 * i] = y[0];
        col[2 * i + 2] = y[1];
    }
    // backward: row i (from NB - 1 down to 1) needs W's record of row i and
    // col[2 (i - 4)]; step t = NB - 1 - i
    double2 Ur[NB][2];
    double nc[NB];
    auto bload = [&](int i) {
        const double2* f = reinterpret_cast<const double2*>(F + brow(i));
        Ur[i][0] = f[0];
        Ur[i][1] = f[1];
        nc[i] = i - 4 >= 0 ? col[2 * (i - 4)] : 0.0;
    };
#pragma unroll
    for (int i = NB - 1; i >= 1; --i)
        if (NB - 1 - i - DB < 0) bload(i);
    double c0 = col[2 * (NB - 1)], c1 = col[2 * (NB - 2)], c2 = col[2 * (NB - 3)], c3 = col[2 * (NB - 4)];
#pragma unroll
    for (int t = 0; t < NB; t += 2) {
#pragma unroll
        for (int u = t + 1; u < NB - 1 && u <= t + 1 + DB; ++u)  // row 0 has nothing above the diagonal: no record
            if (u - DB == t || u - DB == t + 1) bload(NB - 1 - u);
        __builtin_amdgcn_sched_barrier(0);
        double x[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = NB - 1 - t - h;
            x[h] = c0;
            if (i > 0) {
                c0 = c1 - Ur[i][0].x * x[h];
                c1 = c2 - Ur[i][0].y * x[h];
                c2 = c3 - Ur[i][1].x * x[h];
                c3 = nc[i] - Ur[i][1].y * x[h];
            }
        }
        col[2 * (NB - 1 - t)] = x[0];
        col[2 * (NB - 2 - t)] = x[1];
    }
}

// Twisted substitution (image layout and scaling as described at
// solve_twisted): two lanes share a right-hand side, lane `bottom` = 0
// taking rows 0..h+3 from the top, lane 1 rows h..NB-1 from the bottom, the
// pair 32 lanes apart in one wave.  Each lane keeps the register window of
// the one-lane sweeps, walking its rows in its own direction; the two meet in
// the 4 x 4 middle block.  The chains are h and h + 4 rows instead of NB and
// NB - 1.  Reads run DT steps ahead.  (Pairing steps into ds_read2 /
// ds_write2 as the one-lane sweeps do needs a swap of the two values in the
// bottom lane, whose rows run the other way; measured slower.)
template <int NB>
__device__ __forceinline__ void lds_solve_tw(const double* __restrict__ F, double* col, int bottom) {
    constexpr int h = tw_h(NB), DT = 4;
    // sweep step t of phase 1 is row t (top) or NB-1-t (bottom); of phase 3,
    // row h+3-t (top) or h+t (bottom)
    double* c1 = col + (bottom ? 2 * (NB - 1) : 0);
    double* c3 = col + (bottom ? 2 * h : 2 * (h + 3));
    const int dir = bottom ? -2 : 2;  // doubles per phase-1 step (phase 3: the opposite)
    const double* R1 = F + (bottom ? tw_p1b(NB) : 0);
    // ---- phase 1: h steps, four-entry records
    double2 L1[h][2];
    double n1[h];  // right-hand side of sweep row t + 4 (the middle rows at most)
    auto load1 = [&](int t) {
        const double2* f = reinterpret_cast<const double2*>(R1 + 4 * t);
        L1[t][0] = f[0];
        L1[t][1] = f[1];
        n1[t] = c1[dir * (t + 4)];
    };
#pragma unroll
    for (int t = 0; t < DT; ++t) load1(t);
    double b0 = c1[0], b1 = c1[dir], b2 = c1[2 * dir], b3 = c1[3 * dir];
#pragma unroll
    for (int t = 0; t < h; ++t) {
        if (t + DT < h) load1(t + DT);
        __builtin_amdgcn_sched_barrier(0);
        const double y = b0;
        c1[dir * t] = y;
        b0 = b1 - L1[t][0].x * y;
        b1 = b2 - L1[t][0].y * y;
        b2 = b3 - L1[t][1].x * y;
        b3 = n1[t] - L1[t][1].y * y;
    }
    // ---- middle: rows h..h+3 (top lane's b0..b3, bottom lane's b3..b0)
    const double o0 = __shfl_xor(b0, 32), o1 = __shfl_xor(b1, 32), o2 = __shfl_xor(b2, 32), o3 = __shfl_xor(b3, 32);
    const double2* mi = reinterpret_cast<const double2*>(F + tw_mi(NB));
    double r[4];
    {
        const double mine[4] = {b0, b1, b2, b3}, other[4] = {o0, o1, o2, o3};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double top = bottom ? other[k] : mine[k], bot = bottom ? mine[3 - k] : other[3 - k];
            r[k] = top + bot - col[2 * (h + k)];
        }
    }
    double xm[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 m01 = mi[2 * k], m23 = mi[2 * k + 1];
        xm[k] = m01.x * r[0] + m01.y * r[1] + m23.x * r[2] + m23.y * r[3];
    }
    if (!bottom) {
#pragma unroll
        for (int k = 0; k < 4; ++k) col[2 * (h + k)] = xm[k];
    }
    // ---- phase 3: h + 4 steps; the first four take the middle values
    double2 L3[h + 4][4];
    double n3[h + 4];  // right-hand side of sweep row t + 8
    auto load3 = [&](int t) {
        const double* rp = F + (bottom ? tw_p3b_rec(NB, t) : tw_p3a(NB) + 4 * t);
        const double2* f = reinterpret_cast<const double2*>(rp);
        L3[t][0] = f[0];
        L3[t][1] = f[1];
        if (tw_wide(NB, t)) {
            const double2* g = reinterpret_cast<const double2*>(bottom ? rp + 4 : F + tw_z4(NB));
            L3[t][2] = g[0];
            L3[t][3] = g[1];
        }
        n3[t] = t + 8 <= h + 3 ? c3[-dir * (t + 8)] : 0.0;
    };
#pragma unroll
    for (int t = 0; t < DT; ++t) load3(t);
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    double d4 = c3[-dir * 4], d5 = c3[-dir * 5], d6 = c3[-dir * 6], d7 = c3[-dir * 7];
#pragma unroll
    for (int t = 0; t < h + 4; ++t) {
        if (t + DT < h + 4) load3(t + DT);
        __builtin_amdgcn_sched_barrier(0);
        double x;
        if (t < 4) {
            x = bottom ? xm[t] : xm[3 - t];
        } else {
            x = d0;
            c3[-dir * t] = x;
        }
        d0 = d1 - L3[t][0].x * x;
        d1 = d2 - L3[t][0].y * x;
        d2 = d3 - L3[t][1].x * x;
        d3 = d4 - L3[t][1].y * x;
        if (tw_wide(NB, t)) {
            d4 = d5 - L3[t][2].x * x;
            d5 = d6 - L3[t][2].y * x;
            d6 = d7 - L3[t][3].x * x;
            d7 = n3[t] - L3[t][3].y * x;
        } else {
            d4 = d5;
            d5 = d6;
            d6 = d7;
            d7 = n3[t];
        }
    }
}

// LDS DMA (global_load_lds_dwordx4): each active lane loads 16 bytes from
// its own global address into LDS at dst + 16 * lane, without registers.
// dst must be the same for the whole wave.  Completion is tracked by the
// vector-memory counter, so a wave waits with lds_dma_wait() before the data
// is read (and a workgroup barrier publishes it to the other waves).
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;
__device__ __forceinline__ void lds_dma16(const void* src, void* dst_wave) {
    __builtin_amdgcn_global_load_lds((glb_void_t*)src, (lds_void_t*)dst_wave, 16, 0, 0);
}
__device__ __forceinline__ void lds_dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// LDS stride (doubles) of a factor image of FW doubles: FW rounded up to 2
// more than a multiple of 32, so that image o starts 4 o four-byte words
// past a bank boundary.  The substitution lanes of different operators read
// the same row at the same time; with images a whole number of bank periods
// apart those reads would all hit the same four banks.
constexpr int solve_image_lds_stride(int FW) { return FW + (34 - FW % 32) % 32; }

// Copy nimg consecutive factor images of FW doubles each from global memory
// to LDS at a stride of FWP doubles, by DMA: 1 KB per wave instruction, the
// four waves taking alternate kilobytes.  FW * 8 and FWP * 8 are multiples of
// 16 and both ends 16-byte aligned.
template <int FW, int FWP>
__device__ __forceinline__ void dma_images(const double* src, double* dst, int nimg, int w, int lane) {
    constexpr int NB8 = FW * 8, NCH = (NB8 + 1023) >> 10;
    static_assert(NB8 % 16 == 0 && (FWP * 8) % 16 == 0, "16-byte DMA units");
    for (int ch = w; ch < nimg * NCH; ch += 4) {
        const int im = ch / NCH, c = ch - im * NCH;
        const int off = (c << 10) + 16 * lane;
        if (off < NB8)
            lds_dma16(reinterpret_cast<const char*>(src + (size_t)im * FW) + off,
                      reinterpret_cast<char*>(dst + im * FWP) + (c << 10));
    }
}

constexpr int NSLOT = 8;     // modes per workgroup: up to 4 values of m, both signs of k

// 9 weights of one parity for row n, in registers.
struct Row9 {
    double e[W9];
    __device__ __forceinline__ void load(const double* tab, int N, int par, int n) {
#pragma unroll
        for (int j = 0; j < W9; ++j) e[j] = tab[(par * N + n) * W9 + j];
    }
    __device__ __forceinline__ dcplx apply(const dcplx* line, int s0) const {
        dcplx acc = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < W9; ++j) acc = acc + e[j] * line[s0 + j];
        return acc;
    }
};

// One workgroup = 4 waves handles |k| = kabs and GM consecutive m
// (GM = 4, 2, 1 for mp = 1, 2, >= 3 so that the Helmholtz wavenumbers
// mp*m-1 .. mp*m+1 of the block form one contiguous range of <= 6 values,
// shared between neighbouring m).  Slot q = 2 j + s is mode (m0 + j, s ? -k : +k).
// Wave w does the radial-line work of slots 2w, 2w+1 (one lane per radial
// node); wave 0 does the substitutions, one lane per complex right-hand side.
// LDS: the factor area (the pressure images and columns, then the Helmholtz
// images, at a bank-staggered stride), the radial lines (u^n, then the
// right-hand sides and the solution) and the slots' inverse influence
// matrices: about 53 KB at NB = 64, so three workgroups share a compute unit.
// Every input is requested at the start (pressure images and A^-1 by LDS
// DMA, then each slot's u^n and nonlinear terms into registers), and the
// first slot's right-hand side is formed while the second slot's data are
// still arriving; the weights and influence data of later phases are
// requested a phase ahead, and the Helmholtz images follow as soon as the
// pressure images are consumed.
template <typename TNL, int NB, int NW>
__device__ __forceinline__ void k_solve_body(const SolveArgs& a) {
    constexpr int FW = solve_image_doubles(NB, NW);
    constexpr int FWP = solve_image_lds_stride(FW);  // image stride in LDS
    constexpr int XS = NB + 1;         // radial line stride (complex)
    constexpr int FA = NFH * FWP;      // factor area (doubles)
    static_assert(4 * FWP + NSLOT * XS * 2 <= FA, "pressure images and columns fit the factor area");
    __shared__ __align__(16) double sF[FA];
    __shared__ __align__(16) dcplx sX[NSLOT][3][XS];
    // slot q's A^-1 (32 doubles), overwritten by its correction a (8 doubles)
    // once read; the flux correction of (0,0) in slot 0's last entry
    __shared__ __align__(16) double sAi[NSLOT][32];
    double& sGam = sAi[0][31];
    dcplx(*sY)[XS] = reinterpret_cast<dcplx(*)[XS]>(sF + 4 * FWP);  // pressure columns

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
    const int s0r = t.s0[nr];
    const double rinvr = t.rinv[nr];
    const int nfp = min(GM, a.M - m0);
    const int mu_hi = min(mp * (m0 + GM - 1) + 1, a.MU - 1);
    const int nfh = mu_hi - mu_lo + 1;
    const int mw = mp * min(m0 + w, a.M - 1);  // azimuthal wavenumber of this wave's slots
    const size_t ihelm = (size_t)kabs * a.MU + mu_lo;                   // first Helmholtz image
    const size_t ippe = (size_t)a.MU * K + (size_t)kabs * a.M + m0;     // first pressure image

    auto slot_ok = [&](int q) {
        const int j = q >> 1, s = q & 1, mi = m0 + j;
        return j < GM && mi < a.M && (s == 0 || (kabs > 0 && mi > 0));
    };
    auto slot_k = [&](int q) { return (q & 1) ? -kabs : kabs; };
    auto slot_off = [&](int q) {  // offset of row 0 of slot q in one field
        return ((size_t)(m0 + (q >> 1)) * nk + (slot_k(q) + K - 1)) * N;
    };

    // ---- requests, in the order the phases need them: the pressure images
    //      and the slots' A^-1 by LDS DMA, the stencil weights, then slot 2w
    //      and slot 2w+1 (u^n or R and the nonlinear terms, one radial row per
    //      lane) into registers.  The register loads are unconditional (rows
    //      and modes clamped to valid ones), so the counted wait before slot
    //      2w's right-hand side leaves slot 2w+1's loads in flight: loads are
    //      served in order, and slot 2w's right-hand side is formed while
    //      slot 2w+1's data arrive.  The nonlinear-term loads a kind does not
    //      use (N^p for PRED, both for RAW) read one fixed 16-byte location
    //      instead: one cache line for the whole wave, no extra HBM traffic.
    dma_images<FW, FWP>(t.img + ippe * FW, sF, nfp, w, n);
    if (w == 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {  // four slots (16 lanes of 16 bytes each) per instruction
            const int q = 4 * i + (n >> 4);
            if (slot_ok(q))
                lds_dma16(t.ainv + (((size_t)(m0 + (q >> 1)) * nk + (slot_k(q) + K - 1)) * 16) * 2 + 2 * (n & 15),
                          &sAi[4 * i][0]);
        }
    }
    Row9 Lo, Le;  // weights of d2/dr2 + (1/r) d/dr, parity of this wave's m +- 1 and of m
    Lo.load(t.wl, N, (mw + 1) & 1, nr);
    Le.load(t.wl, N, mw & 1, nr);
    const double* src = a.kind == OPF_SOLVE_RAW ? static_cast<const double*>(a.n0) : a.u0;
    const bool use0 = a.kind != OPF_SOLVE_RAW, use1 = a.kind == OPF_SOLVE_CORR;
    const void* nl0 = use0 ? a.n0 : static_cast<const void*>(t.rinv);
    const void* nl1 = use1 ? a.n1 : static_cast<const void*>(t.rinv);
    dcplx ul[2][3];               // u^n (RAW: R) of this lane's row
    vec2<TNL> x0[2][3], x1[2][3];  // N^n and N^p as stored
    auto request = [&](int j) {
        const int q = 2 * w + j;
        const size_t off = ((size_t)min(m0 + (q >> 1), a.M - 1) * nk + (slot_k(q) + K - 1)) * N + nr;
#pragma unroll
        for (int c = 0; c < 3; ++c) ul[j][c] = load_c<double>(src, c * S + off);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x0[j][c] = load_v<TNL>(nl0, use0 ? c * S + off : 0);
            x1[j][c] = load_v<TNL>(nl1, use1 ? c * S + off : 0);
        }
    };
    const auto zero_tail_rows = [&] {  // rows N..NB of this wave's lines stay zero (branch-free substitution)
        for (int i = n; i < 2 * 3 * (XS - N); i += 64) {
            const int j = i / (3 * (XS - N)), rem = i % (3 * (XS - N));
            sX[2 * w + j][rem / (XS - N)][N + rem % (XS - N)] = dcplx{0.0, 0.0};
        }
    };
    request(0);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (sizeof(TNL) == 8) {
        // FP64 nonlinear terms: slot 2w+1 is requested only once slot 2w has
        // arrived.  The launch's load burst is served roughly in the order the
        // requests reach the memory system, so every workgroup then has its
        // first slot by about the middle of the burst and forms that slot's
        // right-hand side before its last data arrive; the workgroups that
        // come last in the order, which set the launch's length, gain most.
        // (With FP32 terms the burst is shorter and this measured slower.)
        zero_tail_rows();
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __builtin_amdgcn_sched_barrier(0);
        request(1);
        __builtin_amdgcn_sched_barrier(0);
    } else {
        request(1);
        __builtin_amdgcn_sched_barrier(0);
        zero_tail_rows();
        // Slot 2w+1's nine loads (nine instructions: the u^n and N^n, N^p
        // reads lie far apart and none is dropped) are the last vector-memory
        // instructions issued: with at most nine outstanding, everything older
        // (the DMA, the weights, slot 2w) has landed.  The compiler's own wait
        // would be vmcnt(0) while the DMA is pending, which would also wait
        // for slot 2w+1.
        __builtin_amdgcn_s_waitcnt(0x0F79);  // vmcnt(9)
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---- R = [1/dt + (1-c) L / Re] u^n + N (+ forcing) in the (+,-,z) form,
    //      slot by slot from this wave's own lines (no workgroup barrier)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int q = 2 * w + j;
        if (n < N) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sX[q][c][n] = ul[j][c];
        }
        __builtin_amdgcn_wave_barrier();
        dcplx rr[3];
        const dcplx ur = ul[j][0], ut = ul[j][1], uz = ul[j][2];
        if (a.kind == OPF_SOLVE_RAW) {
            rr[0] = ur + ix(ut);
            rr[1] = ur - ix(ut);
            rr[2] = uz;
        } else {
            dcplx na[3];  // PRED: N^n; CORR: (1-c) N^n + c N^p
            if (a.kind == OPF_SOLVE_PRED) {
#pragma unroll
                for (int c = 0; c < 3; ++c) na[c] = to_c(x0[j][c]);
            } else {
                const double cc = a.c, c1 = 1.0 - a.c;
#pragma unroll
                for (int c = 0; c < 3; ++c) na[c] = c1 * to_c(x0[j][c]) + cc * to_c(x1[j][c]);
            }
            const int m = mp * (m0 + (q >> 1)), k = slot_k(q);
            const double kap2 = a.alpha * k * a.alpha * k;
            const dcplx dr = Lo.apply(sX[q][0], s0r), dt = Lo.apply(sX[q][1], s0r), dz = Le.apply(sX[q][2], s0r);
            const dcplx up = ur + ix(ut), um = ur - ix(ut);
            const double r2 = rinvr * rinvr;
            const dcplx Lp = (dr + ix(dt)) - (double(m + 1) * double(m + 1) * r2 + kap2) * up;
            const dcplx Lm = (dr - ix(dt)) - (double(m - 1) * double(m - 1) * r2 + kap2) * um;
            const dcplx Lz = dz - (double(m) * double(m) * r2 + kap2) * uz;
            rr[0] = a.inv_dt * up + a.aexp * Lp + (na[0] + ix(na[1]));
            rr[1] = a.inv_dt * um + a.aexp * Lm + (na[0] - ix(na[1]));
            rr[2] = a.inv_dt * uz + a.aexp * Lz + na[2];
            if (m == 0 && k == 0) rr[2].x += a.force;
        }
        __builtin_amdgcn_wave_barrier();  // every lane of the wave has read the u^n lines
        if (n < N && slot_ok(q)) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sX[q][c][n] = rr[c];
            sY[q][n] = 0.5 * (rr[0] + rr[1]);  // R_r, for the divergence
        }
        __builtin_amdgcn_wave_barrier();
    }

    // ---- pressure-Poisson right-hand side div R (P(1) = 0), scaled by 1/U_ii
    {
        Row9 W1o;
        W1o.load(t.d1, N, (mw + 1) & 1, nr);
        const double* dvp = t.dinv + ((size_t)a.MU * K + (size_t)kabs * a.M + min(m0 + w, a.M - 1)) * NB;
        const double dv = n < N ? dvp[n] : 0.0;
        // div R = d/dr R_r + [(1+m) R+ + (1-m) R-] / (2r) + i kappa R_z, R_r = (R+ + R-)/2
        dcplx d[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = 2 * w + j;
            const int m = mp * (m0 + (q >> 1));
            const double kap = a.alpha * slot_k(q);
            d[j] = dcplx{0.0, 0.0};
            if (slot_ok(q) && n < N - 1 && !(m == 0 && kap == 0.0))
                d[j] = W1o.apply(sY[q], s0r) +
                       (0.5 * rinvr) * (double(1 + m) * sX[q][0][n] + double(1 - m) * sX[q][1][n]) +
                       kap * ix(sX[q][2][n]);
        }
        __builtin_amdgcn_wave_barrier();  // every lane of the wave has read the R_r lines
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = 2 * w + j;
            if (n < XS) sY[q][n] = dv * d[j];  // rows N..XS-1 zero (dv = 0 there)
            if (n < XS - 64) sY[q][64 + n] = dcplx{0.0, 0.0};
        }
    }
    lds_dma_wait();  // this wave's share of the pressure images and A^-1 (landed long ago)
    // the next phase's weights and 1/U_ii of H_{m+1}, H_{|m-1|}, H_m at this
    // row, requested now so that they arrive during the substitution
    Row9 W1e;
    W1e.load(t.d1, N, mw & 1, nr);
    const double* dvh = t.dinv + (size_t)kabs * a.MU * NB;
    const double dvp = n < N ? dvh[(size_t)(mw + 1) * NB + n] : 0.0;
    const double dvm = n < N ? dvh[(size_t)abs(mw - 1) * NB + n] : 0.0;
    const double dvz = n < N ? dvh[(size_t)mw * NB + n] : 0.0;
    __syncthreads();
    // The substituting waves run at a raised issue priority: a substitution is
    // one dependent chain per right-hand side, and on a busy compute unit the
    // waves of the other resident workgroups (still forming right-hand sides,
    // their loads having arrived later) would otherwise delay its steps.
    if constexpr (solve_twisted(NB, NW)) {  // right-hand side n & 31, its top lane n < 32
        if (w == 0) {
            __builtin_amdgcn_s_setprio(2);
            if ((n & 31) < 2 * NSLOT && slot_ok((n & 31) >> 1))
                lds_solve_tw<NB>(sF + ((n & 31) >> 2) * FWP, &sY[(n & 31) >> 1][0].x + (n & 1), n >> 5);
            __builtin_amdgcn_s_setprio(0);
        }
    } else if (w == 0) {
        __builtin_amdgcn_s_setprio(2);
        if (n < 2 * NSLOT && slot_ok(n >> 1)) lds_solve<NB, NW>(sF + (n >> 2) * FWP, &sY[n >> 1][0].x + (n & 1));
        __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();

    // ---- R -= grad P, scaled by 1/U_ii of each Helmholtz operator; (0,0):
    //      u_r = 0, real R_theta and R_z.  The Helmholtz images that do not
    //      cover the pressure columns are requested first.
    const int nfh1 = min(nfh, 4);
    dma_images<FW, FWP>(t.img + ihelm * FW, sF, nfh1, w, n);
    {
        if (n < N) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int q = 2 * w + j;
                if (!slot_ok(q)) continue;
                const int m = mp * (m0 + (q >> 1));
                const double kap = a.alpha * slot_k(q);
                dcplx r0 = sX[q][0][n], r1 = sX[q][1][n], r2 = sX[q][2][n];
                const dcplx P = sY[q][n];
                if (a.p_out && !(m == 0 && kap == 0.0))  // the pressure head before the influence correction
                    store_c<double>(a.p_out, slot_off(q) + n, P);
                if (n == N - 1) {
                    r0 = r1 = r2 = dcplx{0.0, 0.0};
                    if (m == 0 && kap == 0.0 && a.wall) {  // (0,0): Dirichlet values u_theta(1), u_z(1)
                        const size_t w0 = (size_t)(K - 1) * 2, ws = (size_t)a.M * nk * 2;
                        r0 = dcplx{a.wall[ws + w0], 0.0};
                        r2 = dcplx{a.wall[2 * ws + w0], 0.0};
                    }
                } else if (m == 0 && kap == 0.0) {
                    const dcplx d = r0 - r1;  // 2 i R_theta
                    r0 = dcplx{0.5 * d.y, 0.0};
                    r1 = dcplx{0.0, 0.0};
                    r2 = dcplx{r2.x, 0.0};
                } else {
                    const dcplx dP = W1e.apply(sY[q], s0r);
                    const dcplx mP = (double(m) * rinvr) * P;
                    r0 = r0 - (dP - mP);
                    r1 = r1 - (dP + mP);
                    r2 = r2 - kap * ix(P);
                }
                // (0,0) solves u_theta with H_1 in the + slot and u_z with H_0
                sX[q][0][n] = dvp * r0;
                sX[q][1][n] = dvm * r1;
                sX[q][2][n] = dvz * r2;
            }
        }
    }
    __syncthreads();  // the pressure columns are read: the rest of the Helmholtz images may land there
    if (nfh > nfh1)
        dma_images<FW, FWP>(t.img + (ihelm + nfh1) * FW, sF + nfh1 * FWP, nfh - nfh1, w, n);
    lds_dma_wait();
    // influence data of this wave's m (one radial row per lane), requested
    // before the substitution and used after it
    double hv[NHOM];
    {
        const double* h = t.hom + ((size_t)min(m0 + w, a.M - 1) * K + kabs) * NHOM * N;
#pragma unroll
        for (int j = 0; j < NHOM; ++j) hv[j] = h[j * N + nr];
    }
    __syncthreads();
    if constexpr (solve_twisted(NB, NW)) {  // right-hand side 32 w + (n & 31), waves 0 and 1
        const int rh = 32 * w + (n & 31);
        if (w < 2) {
            __builtin_amdgcn_s_setprio(2);
            if (rh < 6 * NSLOT) {
                const int q = rh / 6, c = (rh >> 1) % 3;
                if (slot_ok(q)) {
                    const int m = mp * (m0 + (q >> 1));
                    const int mu = c == 0 ? m + 1 : (c == 1 ? abs(m - 1) : m);
                    lds_solve_tw<NB>(sF + (mu - mu_lo) * FWP, &sX[q][c][0].x + (rh & 1), n >> 5);
                }
            }
            __builtin_amdgcn_s_setprio(0);
        }
    } else if (w == 0) {
        __builtin_amdgcn_s_setprio(2);
        if (n < 6 * NSLOT) {
            const int q = n / 6, c = (n >> 1) % 3;
            if (slot_ok(q)) {
                const int m = mp * (m0 + (q >> 1));
                const int mu = c == 0 ? m + 1 : (c == 1 ? abs(m - 1) : m);
                lds_solve<NB, NW>(sF + (mu - mu_lo) * FWP, &sX[q][c][0].x + (n & 1));
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    // ---- influence matrix a = -A^{-1} g(u_b); fixed flux on (0,0) --------
    if (w == 1 && m0 == 0 && kabs == 0) {  // (0,0): flux of u_z,b over the radial quadrature
        double qs = n < N ? t.quad[n] * sX[0][2][n].x : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) qs += __shfl_xor(qs, o, 64);
        if (n == 0) {
            const double gamma = a.fixed_flux ? (0.25 - qs) * t.qG_inv : 0.0;
            sGam = gamma;
            if (a.beta_out) *a.beta_out = gamma * a.Re * 0.25;
        }
    }
    if (tid < NSLOT && slot_ok(tid)) {
        const int q = tid;
        const int mi = m0 + (q >> 1), m = mp * mi, k = slot_k(q);
        if (m == 0 && k == 0) {
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
            const double* A = sAi[q];
            dcplx av[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dcplx acc = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc = acc + cm(dcplx{A[2 * (4 * i + j)], A[2 * (4 * i + j) + 1]}, g[j]);
                av[i] = dcplx{-acc.x, -acc.y};
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) reinterpret_cast<dcplx*>(sAi[q])[i] = av[i];
        }
    }
    __syncthreads();
    Row9 W1o, W1v;  // first-derivative weights of this lane's row, parities of m +- 1 and m (vorticity)
    W1o.load(t.d1, N, (mw + 1) & 1, nr);
    W1v.load(t.d1, N, mw & 1, nr);
    if (n < N) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = 2 * w + j;
            if (!slot_ok(q)) continue;
            const int mi = m0 + (q >> 1), m = mp * mi, k = slot_k(q);
            const size_t off = slot_off(q) + n;
            const bool mirror = (mi == 0 && kabs > 0);  // m = 0: -k is the conjugate of +k
            const size_t offc = ((size_t)mi * nk + (K - 1 - kabs)) * N + n;
            dcplx up = sX[q][0][n], um = sX[q][1][n], uz = sX[q][2][n];
            if (m == 0 && k == 0) {
                const double ut = up.x;
                uz = dcplx{uz.x + sGam * t.green[n], 0.0};
                up = dcplx{0.0, ut};
                um = dcplx{0.0, -ut};
            } else {
                const double kap = a.alpha * k;
                const double h1p = hv[0], h1m = hv[1], qv = hv[2], h2 = hv[3], h3 = hv[4], h4 = hv[5], P1 = hv[6];
                const dcplx* sa = reinterpret_cast<const dcplx*>(sAi[q]);
                const dcplx a1 = sa[0], a2 = sa[1], a3 = sa[2], a4 = sa[3];
                up = up + h1p * a1 + h2 * a2;
                um = um + h1m * a1 + h3 * a3;
                uz = uz - (kap * qv) * ix(a1) + h4 * a4;  // h1: u_z = -i kappa q
                if (a.p_out) {
                    const dcplx pp = load_c<double>(a.p_out, off) + P1 * a1;
                    store_c<double>(a.p_out, off, pp);
                    if (mirror) store_c<double>(a.p_out, offc, dcplx{pp.x, -pp.y});
                }
            }
            // ---- output u (r, theta, z); omega from the stored components
            const dcplx ur = 0.5 * (up + um), ut = 0.5 * dcplx{(up - um).y, -(up - um).x};
            const dcplx uo[3] = {ur, ut, uz};
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
            if (a.p_out && m == 0 && k == 0) store_c<double>(a.p_out, off, dcplx{0.0, 0.0});
            // omega is computed from (u_r, u_theta, u_z) as stored, so it
            // equals what the standalone vorticity kernel gives for the same state
            sX[q][0][n] = ur;
            sX[q][1][n] = ut;
            sX[q][2][n] = uz;
        }
    }
    // the vorticity stencils read only this wave's own lines: a wave-level
    // ordering suffices (no wait for the stores above)
    __builtin_amdgcn_wave_barrier();
    if (a.w_out && n < N) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = 2 * w + j;
            if (!slot_ok(q)) continue;
            const int mi = m0 + (q >> 1), m = mp * mi, k = slot_k(q);
            const bool mirror = (mi == 0 && kabs > 0);
            dcplx wo[3];
            curl_row(W1v.apply(sX[q][2], s0r), W1o.apply(sX[q][1], s0r), rinvr, m, a.alpha * k, sX[q][0][n],
                     sX[q][1][n], sX[q][2][n], wo[0], wo[1], wo[2]);
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

// Three workgroups (12 waves) per compute unit where the LDS allows it (all
// but the last nine rows narrow: about 53 KB at NB = 64), so at most 168
// VGPRs; otherwise two.
constexpr int solve_waves(int NB, int NW) { return NW == NB - 9 ? 3 : 2; }
template <typename TNL, int NB, int NW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(solve_waves(NB, NW), solve_waves(NB, NW))))
void k_solve(SolveArgs a) {
    k_solve_body<TNL, NB, NW>(a);
}
template <typename TNL, int NB, int NW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(solve_waves(NB, NW), solve_waves(NB, NW))))
void k_solve_b(const SolveArgs* __restrict__ aa) {
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
        sL[0][n] = load_c<double>(a.u, off);
        sL[1][n] = load_c<double>(a.u, S + off);
        sL[2][n] = load_c<double>(a.u, 2 * S + off);
    }
    __syncthreads();
    if (n < N) {
        const int s0 = a.t.s0[n];
        Row9 de, dod;
        de.load(a.t.d1, N, m & 1, n);
        dod.load(a.t.d1, N, (m + 1) & 1, n);
        dcplx wo[3];
        curl_row(de.apply(sL[2], s0), dod.apply(sL[1], s0), a.t.rinv[n], m, a.alpha * (kk - (K - 1)), sL[0][n],
                 sL[1][n], sL[2][n], wo[0], wo[1], wo[2]);
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

static hipError_t launch_solve_any(const SolveArgs& a, const SolveArgs* batch, int members, int precision,
                                   hipStream_t s, const KernelTiming& kt) {
    const bool b = batch != nullptr;
    const dim3 grid(a.K * ((a.M + a.gm - 1) / a.gm), b ? members : 1), block(256);
    // NB rows and NW narrow rows as the factor images were written
    // (solve_nb, solve_nw); the members of a batch share N and with it both
#define OPF_SOLVE_LAUNCH(TNL, NB, NW)                                                   \
    if (b) hipLaunchKernelGGL((k_solve_b<TNL, NB, NW>), grid, block, 0, s, batch); \
    else launch_timed((k_solve<TNL, NB, NW>), grid, block, 0, s, kt, a);
#define OPF_SOLVE_NW(TNL, NB)                                                       \
    if (solve_nw(a.N, a.narrow) == NB - 9) { OPF_SOLVE_LAUNCH(TNL, NB, NB - 9) }   \
    else if (solve_nw(a.N, a.narrow) == NB - 25) { OPF_SOLVE_LAUNCH(TNL, NB, NB - 25) } \
    else { OPF_SOLVE_LAUNCH(TNL, NB, 0) }
    if (solve_nb(a.N) == 32) {
        if (precision == OPF_MIXED) { OPF_SOLVE_NW(float, 32) }
        else { OPF_SOLVE_NW(double, 32) }
    } else if (solve_nb(a.N) == 48) {
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

hipError_t launch_solve_batch(const SolveArgs& a, const SolveArgs* batch, int members, int precision,
                              hipStream_t s) {
    return launch_solve_any(a, batch, members, precision, s, KernelTiming{});
}

hipError_t launch_solve(const SolveArgs& a, int precision, hipStream_t s, const KernelTiming& kt) {
    return launch_solve_any(a, nullptr, 1, precision, s, kt);
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
