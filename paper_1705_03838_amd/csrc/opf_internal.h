// Internal definitions shared by the host code and the HIP kernels of the
// pipe-flow time-step library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/opf.h"

namespace opf {

constexpr int W9 = 9;     // finite-difference stencil width (Section 2: 9 points)
constexpr int HALF = 4;   // points on each side of a centred stencil
constexpr int FACW = 14;  // doubles per LU factor row: 8 of L, 4 of U, 1/U_ii, pad
// In HBM the N rows of one factor are FMAIN-double main records (L[i+1..i+4][i],
// U[i-1..i-4][i], 1/U_ii, pad) followed by FTAIL-double tail records
// (L[i+5..i+8][i]), N FACW doubles in all; in LDS a row is one FACW record
// (L[i+1..i+8][i], U[i-1..i-4][i], 1/U_ii, pad).
constexpr int FMAIN = 10;
constexpr int FTAIL = 4;
constexpr int NHOM = 7;   // real radial lines of influence data per (m,|k|)
// Substitution images of the LU factors (see solve_image_doubles): with
// A = L U = L D W (D = diag U, W unit upper), A x = b is solved as
// (D^-1 L D) y = D^-1 b, then W x = y.  Per operator, padded to NB rows:
// the forward part, row i holding Lh[i+1..i+4][i] for i < NW and
// Lh[i+1..i+8][i] from NW on (Lh = D^-1 L D), then the backward part, row
// i >= 1 holding W[i-1..i-4][i] at solve_image_fwd + 4 (i - 1) (row 0 has no
// entries above the diagonal); rows N..NB-1 are zero.  dinv = 1/U_ii per row.
__host__ __device__ constexpr int solve_image_fwd(int NB, int NW) { return 4 * NW + 8 * (NB - NW); }
__host__ __device__ constexpr int solve_image_doubles(int NB, int NW) { return solve_image_fwd(NB, NW) + 4 * (NB - 1); }
// Twisted substitution images, used where NW = NB - 9 (then N = NB: the
// clamped wall stencils put the first column with more than four entries
// below the diagonal at N - 9).  The operator is eliminated from both ends
// without pivoting: columns 0..h-1 top-down, columns NB-1..h+4 bottom-up,
// h = (NB - 4) / 2, which leaves rows h..h+3 coupled only among themselves.
// With p_i the pivots of the top and bottom rows and s_i = 1/p_i there (1 on
// the middle rows), the right-hand side arrives scaled by s (dinv = s), and
// a top lane and a bottom lane solve together:
//   phase 1, h steps each: the top lane runs down rows 0..h-1, the bottom
//     lane up rows NB-1..h+4, each record holding the four scaled
//     multipliers s_i l_ij p_j of its column (rows below, resp. above);
//   middle: both lanes add their four remainders for rows h..h+3, subtract
//     the right-hand side once and apply Mi, the inverse of the middle block;
//   phase 3, h + 4 steps each: the top lane runs up columns h+3..0, the
//     bottom lane down columns h..NB-1 (the first four steps with the middle
//     values known), records holding s_i A~[i][j] for the rows of its own
//     part: four entries, eight for the bottom columns NB-9..NB-7 (the top
//     lane reads four zeros there).
// Layout per operator (doubles): phase-1 top records, phase-1 bottom
// records, Mi (16, row-major), four zeros, phase-3 top records, phase-3
// bottom records; 8 NB + 32 in all, the size of the standard image with
// NW = NB - 9.
__host__ __device__ constexpr bool solve_twisted(int NB, int NW) { return NW == NB - 9; }
__host__ __device__ constexpr int tw_h(int NB) { return (NB - 4) / 2; }
__host__ __device__ constexpr int tw_p1b(int NB) { return 4 * tw_h(NB); }
__host__ __device__ constexpr int tw_mi(int NB) { return 8 * tw_h(NB); }
__host__ __device__ constexpr int tw_z4(int NB) { return tw_mi(NB) + 16; }
__host__ __device__ constexpr int tw_p3a(int NB) { return tw_z4(NB) + 4; }
__host__ __device__ constexpr int tw_p3b(int NB) { return tw_p3a(NB) + 4 * (tw_h(NB) + 4); }
// first of the three wide phase-3 steps of the bottom lane (columns NB-9..NB-7)
__host__ __device__ constexpr int tw_w0(int NB) { return NB - 9 - tw_h(NB); }
__host__ __device__ constexpr bool tw_wide(int NB, int t) { return t >= tw_w0(NB) && t < tw_w0(NB) + 3; }
// offset of the bottom lane's phase-3 record of step t
__host__ __device__ constexpr int tw_p3b_rec(int NB, int t) {
    return tw_p3b(NB) + 4 * t + 4 * ((t < tw_w0(NB) ? tw_w0(NB) : (t > tw_w0(NB) + 3 ? tw_w0(NB) + 3 : t)) - tw_w0(NB));
}
static_assert(tw_p3b_rec(64, tw_h(64) + 4) == solve_image_doubles(64, 55), "twisted image size, NB = 64");
static_assert(tw_p3b_rec(48, tw_h(48) + 4) == solve_image_doubles(48, 39), "twisted image size, NB = 48");
static_assert(tw_p3b_rec(32, tw_h(32) + 4) == solve_image_doubles(32, 23), "twisted image size, NB = 32");
// Padded row count and narrow-row count of the substitution for N radial
// points whose LU columns j < narrow have at most four entries below the
// diagonal: NB = 32, 48 or 64, NW = NB - 9, NB - 25 or 0 (the largest the
// bound allows).
__host__ __device__ constexpr int solve_nb(int N) { return N <= 32 ? 32 : (N <= 48 ? 48 : 64); }
__host__ __device__ constexpr int solve_nw(int N, int narrow) {
    return narrow >= solve_nb(N) - 9 ? solve_nb(N) - 9 : (narrow >= solve_nb(N) - 25 ? solve_nb(N) - 25 : 0);
}
constexpr int NMAX = 64;  // radial points handled by one solve workgroup

// Complex number used by the kernels (interleaved re/im, same layout as
// complex128 / complex64 in memory).  Aligned to its full size so that one
// value is one 16-byte (FP64) or 8-byte (FP32) load or store, in HBM and LDS.
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

// Device-resident tables built at create time (all pointers into the
// caller's workspace).
struct Tables {
    const double* r;      // [N] radial nodes
    const double* rinv;   // [N] 1/r
    const double* quad;   // [N] weights of int_0^1 g(r) r dr (g even in r)
    const double* d1;     // [2][N][9] folded first-derivative weights, parity 0 even / 1 odd
    const double* d2;     // [2][N][9] folded second-derivative weights
    const int* s0;        // [N] first column of row n's 9-point window
    const double* fac;    // [nfac] banded LU factors of N FACW doubles (main then tail records)
    const double* img;    // substitution images: [K][MU] Helmholtz, then [K][M] pressure
    const double* dinv;   // [K][MU] then [K][M] rows of NB values: 1/U_ii (0 past N)
    const double* wl;     // [2][N][9] folded weights of d2/dr2 + (1/r) d/dr, parity 0 even / 1 odd
    const double* hom;    // [M][K][NHOM][N] influence data (h1+, h1-, q, h2, h3, h4, P1)
    const double* ainv;   // [M][2K-1][16][2] inverse influence matrices (complex)
    const double* green;  // [N] flux Green's function: H_0 u_G = 1, u_G(1) = 0
    double qG_inv;        // 1 / int_0^1 u_G r dr
};

// Arguments of one nonlinear-term evaluation (three transform kernels).
struct NLArgs {
    int N, M, K, nk;
    const void* in[6];  // spectral u_r,u_t,u_z,w_r,w_t,w_z  [M][nk][N] (storage type)
    void* H;            // z-transformed fields [6][N][M][3K] (compute type)
    void* G;            // theta-transformed products [3][N][M][3K] (compute type)
    void* out[3];       // spectral N_r, N_t, N_z [M][nk][N] (storage type)
    const void* twz;    // e^{-2 pi i t / 3K}, t < 3K (compute type)
    const void* twt;    // e^{-2 pi i t / 3M}, t < 3M (compute type)
    double scale;       // 1 / (9 K M)
    double rot[3];      // rotation vector Omega (Cartesian, z the pipe axis) of the Coriolis force
    int rotating;       // nonzero: add -2 Omega x u to u x omega (mp = 1 unless Omega is axial)
    int tz;             // axial points per theta-stage workgroup (tile shape), see tz_ok
    int ztile;          // radial lines per z-transform workgroup (tile shape), see ztile_ok
};

// Arguments of one substep solve (one kernel).
struct SolveArgs {
    int N, M, K, nk, mp, MU;
    int gm;             // consecutive m per workgroup (tile shape), see gm_ok
    int narrow;         // LU columns j < narrow have L[i][j] = 0 for i > j + 4
    int kind;           // OPF_SOLVE_PRED / CORR / RAW
    int fixed_flux;
    double alpha, Re, c, inv_dt, aexp, force;
    const double* u0;   // u^n (external layout, complex128); PRED / CORR
    const void* n0;     // N^n (nonlinear storage type), or R (complex128) for RAW
    const void* n1;     // N^p for CORR
    double* u_out;      // complex128 output state (nullable)
    float* u_out32;     // complex64 shadow of the output state (nullable)
    void* w_out;        // vorticity of the output (nonlinear storage type, nullable)
    double* p_out;      // pressure head [M][nk][N] complex128 (nullable)
    double* beta_out;   // flux correction beta (device scalar)
    const double* wall; // wall velocity [3][M][nk] complex (r, theta, z) at r = 1, or null (no slip)
    Tables t;
};

// Arguments of the vorticity / diagnostics kernels.
struct AuxArgs {
    int N, M, K, nk, mp;
    int mirror;         // vorticity: m = 0, k < 0 written as conjugates of k > 0
    double alpha;
    const double* u;    // complex128 external layout
    double* w;          // complex128 output (vorticity)
    double* partial;    // [M][2] per-m sums of |u|^2 and |omega|^2 (quadrature weighted)
    const double* wall; // wall velocity as in SolveArgs, or null
    Tables t;
};

// Arguments of the operator-table kernels (banded LU factors, influence
// data, flux Green's function), written into the workspace tables.
struct FactorArgs {
    int N, M, K, MU, mp;
    double alpha;
    double cr;          // c / Re
    double inv_dt;      // 1 / dt
    const double* rinv;
    const double* quad;
    const double* d1;
    const double* d2;
    const int* s0;
    double* fac;        // [MU K + M K] factors of N FACW doubles: H_{|mu|,|k|} then L_{m,|k|}
    double* img;        // substitution images (Tables::img), NB rows, NW narrow rows
    double* dinv;       // Tables::dinv
    int NB, NW;
    double* hom;        // [M][K][NHOM][N]
    double* ainv;       // [M][2K-1][16][2]
    double* green;      // [N]
    int* flags;         // [MU K + M K] factor status, then [M (2K-1)] influence status
    double* qg;         // int_0^1 u_G r dr (device scalar)
};
// Factor the Helmholtz operators (and, with pressure, the pressure
// operators and the unit-wall pressure P1), then the homogeneous solutions,
// inverse influence matrices and Green's function.
hipError_t launch_operator_tables(const FactorArgs& a, bool pressure, hipStream_t s);

// Kernel-only timing of one launch: when start is set, the launch goes
// through hipExtLaunchKernelGGL, which records start and stop around the
// kernel itself (no dispatch gap), for opf_profile_steps.
struct KernelTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
template <typename... Args, typename F = void (*)(Args...)>
inline void launch_timed(F kernel, const dim3& grid, const dim3& block, uint32_t lds, hipStream_t s,
                         const KernelTiming& kt, Args... args) {
    if (kt.start) hipExtLaunchKernelGGL(kernel, grid, block, lds, s, kt.start, kt.stop, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// Launchers (return the first HIP error).
hipError_t launch_nonlinear(const NLArgs& a, int precision, hipStream_t s);
// One of the three transform kernels: 0 z-inverse, 1 theta + product, 2 z-forward.
hipError_t launch_nonlinear_stage(const NLArgs& a, int precision, int stage, hipStream_t s,
                                  const KernelTiming& kt = KernelTiming{});
bool nonlinear_supported(int M, int K);
// Admissible transform tile shapes: tz in {2, 4, 8} axial points per theta
// workgroup, zt in {4, 8, 16} radial lines per z workgroup, each while the
// longer radix pass fits the workgroup.
bool tz_ok(int tz, int M);
bool ztile_ok(int zt, int K);
constexpr int DEFAULT_TZ = 4, DEFAULT_ZTILE = 8;
// Radial lines per z workgroup before any tuning: 16 with FP32 transforms
// (half the bytes per line, so the same bytes per workgroup as 8 lines in
// FP64), else 8.
inline int default_ztile(int precision) { return precision == OPF_MIXED ? 16 : DEFAULT_ZTILE; }
hipError_t launch_solve(const SolveArgs& a, int precision, hipStream_t s, const KernelTiming& kt = KernelTiming{});
// Batched forms: one launch for `members` argument records in device memory
// (grid.y = member); `proto` gives the shared sizes.
hipError_t launch_nonlinear_batch(const NLArgs& proto, const NLArgs* dev_args, int members, int precision,
                                  int stage, hipStream_t s);
hipError_t launch_solve_batch(const SolveArgs& proto, const SolveArgs* dev_args, int members, int precision,
                              hipStream_t s);
int default_gm(int mp);
bool gm_ok(int gm, int mp);
constexpr int NFH = 6;  // Helmholtz factors a solve workgroup stages at once
hipError_t launch_vorticity(const AuxArgs& a, hipStream_t s);
hipError_t launch_energy(const AuxArgs& a, hipStream_t s);
// Per mode q: part[2q] = max |g| of (u+(1), u-(1), u_z(1), div u(1)),
// part[2q+1] = max over interior nodes of |div u|.
hipError_t launch_divg(const AuxArgs& a, double* part, hipStream_t s);
// Largest |u_r| wr[n] + |u_theta| wt[n] + |u_z| wz over the physical points
// of each (n, 4-point z tile) workgroup into out[block], from the
// z-transformed fields in a.H (stage 0 of the nonlinear term).
hipError_t launch_cfl(const NLArgs& a, int precision, const double* wr, const double* wt, double wz, double* out,
                      hipStream_t s);

// Context accessors for translation units other than the host core.
hipStream_t ctx_stream(const opf_ctx* c);
const opf_params& ctx_params(const opf_ctx* c);
void ctx_set_error(opf_ctx* c, const std::string& msg);

}  // namespace opf
