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
//   k_theta : per (n, 8 axial points): the 6 fields' M azimuthal coefficients
//             are packed two real fields per complex line, inverse FFT over
//             3M points, u x omega at every point, forward FFT of
//             (N_r + i N_t) and (N_z + i 0), unpacked and scaled by 1/(9KM)
//             into G[comp][n][m][z].  Physical fields never leave LDS.
//   k_zfwd  : per (comp, m, 8 radial nodes): forward c2c over 3K points,
//             |k| < K kept, written to the spectral layout.
//
// FFTs are radix-4/2/3 Stockham passes on lines held in LDS, each pass
// staged through registers (read all, barrier, write all), with FP64 (or
// FP32) twiddles from a host-built table staged in LDS.
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

__host__ __device__ constexpr int count2(int L) { int c = 0; while (L % 2 == 0) { L /= 2; ++c; } return c; }
__host__ __device__ constexpr int count3(int L) { int c = 0; while (L % 3 == 0) { L /= 3; ++c; } return c; }
template <int L>
__host__ __device__ constexpr int n_stages() { return count2(L) / 2 + count2(L) % 2 + count3(L); }
template <int L>
__host__ __device__ constexpr int radix_of(int s) {
    return s < count2(L) / 2 ? 4 : (s < count2(L) / 2 + count2(L) % 2 ? 2 : 3);
}

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

// One Stockham pass of radix R over NLINE lines of length L (stride LS) in
// LDS; NS = product of the radices of the previous passes.
template <typename T, int L, int NLINE, int LS, int NT, int R, int NS>
__device__ __forceinline__ void fft_pass(cpx<T>* buf, const cpx<T>* tw, int sign) {
    constexpr int NB = NLINE * (L / R);
    constexpr int PER = (NB + NT - 1) / NT;
    constexpr int TWS = L / (NS * R);
    cpx<T> v[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * NT;
        if (NB % NT == 0 || b < NB) {
            const int line = b / (L / R), j = b % (L / R);
            const cpx<T>* x = buf + line * LS;
            const int k = j % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cpx<T> a = x[j + r * (L / R)];
                if (NS > 1 && r > 0) {
                    const cpx<T> w = tw[k * r * TWS];
                    a = sign < 0 ? cmul(a, w) : cmulc(a, w);
                }
                v[p][r] = a;
            }
            dft<T, R>(v[p], sign);
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * NT;
        if (NB % NT == 0 || b < NB) {
            const int line = b / (L / R), j = b % (L / R);
            cpx<T>* x = buf + line * LS;
            const int k = j % NS;
            const int o = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) x[o + r * NS] = v[p][r];
        }
    }
    __syncthreads();
}

template <typename T, int L, int NLINE, int LS, int NT, int S, int NS>
struct FFTStages {
    static __device__ __forceinline__ void run(cpx<T>* buf, const cpx<T>* tw, int sign) {
        if constexpr (S < n_stages<L>()) {
            constexpr int R = radix_of<L>(S);
            fft_pass<T, L, NLINE, LS, NT, R, NS>(buf, tw, sign);
            FFTStages<T, L, NLINE, LS, NT, S + 1, NS * R>::run(buf, tw, sign);
        }
    }
};

// Unnormalised DFT of NLINE lines in LDS, in place:
// sign -1: X_q = sum_j x_j e^{-2 pi i jq/L};  sign +1: e^{+2 pi i jq/L}.
template <typename T, int L, int NLINE, int LS, int NT>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, const cpx<T>* tw, int sign) {
    FFTStages<T, L, NLINE, LS, NT, 0, 1>::run(buf, tw, sign);
}

template <typename TO, typename TI>
__device__ __forceinline__ cpx<TO> cvt(cpx<TI> a) { return {TO(a.x), TO(a.y)}; }

constexpr int NT = 256;

// ---------------------------------------------------------------------------
// k_zinv: spectral [M][nk][N] -> H[f][n][m][z], z = 0..3K-1.
template <typename TS, typename T, int L>
__global__ __launch_bounds__(NT) void k_zinv(NLArgs a) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);  // [TILE][L]
    cpx<T>* tw = buf + TILE * L;                        // [L]
    const int N = a.N, M = a.M, K = a.K, nk = a.nk;
    const int ntile = (N + TILE - 1) / TILE;
    const int tile = blockIdx.x % ntile;
    const int m = (blockIdx.x / ntile) % M;
    const int f = blockIdx.x / (ntile * M);
    const int n0 = tile * TILE;
    const int tid = threadIdx.x;
    const cpx<T>* twg = reinterpret_cast<const cpx<T>*>(a.twz);
    for (int t = tid; t < L; t += NT) tw[t] = twg[t];
    const cpx<TS>* src = reinterpret_cast<const cpx<TS>*>(a.in[f]) + (size_t)m * nk * N;
    // bin-major fill, radial node fastest: coalesced reads of each k row
    for (int t = tid; t < TILE * L; t += NT) {
        const int bin = t / TILE, nn = t % TILE, n = n0 + nn;
        cpx<T> v = {T(0), T(0)};
        int kk = -1;
        if (bin < K) kk = bin + K - 1;
        else if (bin > L - K) kk = bin - L + K - 1;
        if (kk >= 0 && n < N) v = cvt<T>(src[(size_t)kk * N + n]);
        buf[nn * L + bin] = v;
    }
    __syncthreads();
    lds_fft<T, L, TILE, L, NT>(buf, tw, +1);
    cpx<T>* dst = reinterpret_cast<cpx<T>*>(a.H) + (size_t)f * N * M * L;
    for (int t = tid; t < TILE * L; t += NT) {
        const int nn = t / L, z = t % L, n = n0 + nn;
        if (n < N) dst[((size_t)n * M + m) * L + z] = buf[t];
    }
}

// ---------------------------------------------------------------------------
// k_theta: per (n, TILE axial points): inverse theta FFTs of the six fields
// (two real fields per complex line), u x omega, forward FFTs, unpack.
template <typename T, int L>
__global__ __launch_bounds__(NT) void k_theta(NLArgs a) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);  // [3][TILE][L]
    cpx<T>* tw = buf + 3 * TILE * L;                    // [L]
    const int N = a.N, M = a.M, L3K = 3 * a.K;
    const int nzt = (L3K + TILE - 1) / TILE;
    const int n = blockIdx.x / nzt;
    const int z0 = (blockIdx.x % nzt) * TILE;
    const int tid = threadIdx.x;
    const cpx<T>* twg = reinterpret_cast<const cpx<T>*>(a.twt);
    for (int t = tid; t < L; t += NT) tw[t] = twg[t];
    const cpx<T>* H = reinterpret_cast<const cpx<T>*>(a.H);
    const size_t fstride = (size_t)N * M * L3K;
    // pack pairs (u_r,u_t), (u_z,w_r), (w_t,w_z): Z = A + iB on m >= 0 and
    // conj(A) + i conj(B) on bins L-m; zero elsewhere
    for (int t = tid; t < 3 * L * TILE; t += NT) {
        const int p = t / (L * TILE);
        const int rem = t % (L * TILE);
        const int j = rem / TILE, zz = rem % TILE, z = z0 + zz;
        cpx<T> v = {T(0), T(0)};
        int m = -1;
        bool neg = false;
        if (j < M) m = j;
        else if (j > L - M) { m = L - j; neg = true; }
        if (m >= 0 && z < L3K) {
            const size_t off = ((size_t)n * M + m) * L3K + z;
            const cpx<T> A = H[(2 * p) * fstride + off];
            const cpx<T> B = H[(2 * p + 1) * fstride + off];
            v = neg ? cpx<T>{A.x + B.y, B.x - A.y} : cpx<T>{A.x - B.y, A.y + B.x};
        }
        buf[(p * TILE + zz) * L + j] = v;
    }
    __syncthreads();
    lds_fft<T, L, 3 * TILE, L, NT>(buf, tw, +1);
    for (int t = tid; t < TILE * L; t += NT) {
        const int zz = t / L, j = t % L;
        const cpx<T> c0 = buf[(0 * TILE + zz) * L + j];
        const cpx<T> c1 = buf[(1 * TILE + zz) * L + j];
        const cpx<T> c2 = buf[(2 * TILE + zz) * L + j];
        const T ur = c0.x, ut = c0.y, uz = c1.x, wr = c1.y, wt = c2.x, wz = c2.y;
        buf[(0 * TILE + zz) * L + j] = {ut * wz - uz * wt, uz * wr - ur * wz};
        buf[(1 * TILE + zz) * L + j] = {ur * wt - ut * wr, T(0)};
    }
    __syncthreads();
    lds_fft<T, L, 2 * TILE, L, NT>(buf, tw, -1);
    cpx<T>* G = reinterpret_cast<cpx<T>*>(a.G);
    const T h = T(0.5) * T(a.scale);
    for (int t = tid; t < M * TILE; t += NT) {
        const int m = t / TILE, zz = t % TILE, z = z0 + zz;
        if (z >= L3K) continue;
        const int mc = m == 0 ? 0 : L - m;
        const cpx<T> Z0 = buf[(0 * TILE + zz) * L + m], Y0 = buf[(0 * TILE + zz) * L + mc];
        const cpx<T> Z1 = buf[(1 * TILE + zz) * L + m], Y1 = buf[(1 * TILE + zz) * L + mc];
        const size_t off = ((size_t)n * M + m) * L3K + z;
        // A = (Z + conj Y)/2, B = (Z - conj Y)/(2i)
        G[off] = {h * (Z0.x + Y0.x), h * (Z0.y - Y0.y)};
        G[fstride + off] = {h * (Z0.y + Y0.y), h * (Y0.x - Z0.x)};
        G[2 * fstride + off] = {h * (Z1.x + Y1.x), h * (Z1.y - Y1.y)};
    }
}

// ---------------------------------------------------------------------------
// k_zfwd: G[f][n][m][z] -> spectral [M][nk][N], |k| < K kept.
template <typename TS, typename T, int L>
__global__ __launch_bounds__(NT) void k_zfwd(NLArgs a) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);  // [TILE][L]
    cpx<T>* tw = buf + TILE * L;
    const int N = a.N, M = a.M, K = a.K, nk = a.nk;
    const int ntile = (N + TILE - 1) / TILE;
    const int tile = blockIdx.x % ntile;
    const int m = (blockIdx.x / ntile) % M;
    const int f = blockIdx.x / (ntile * M);
    const int n0 = tile * TILE;
    const int tid = threadIdx.x;
    const cpx<T>* twg = reinterpret_cast<const cpx<T>*>(a.twz);
    for (int t = tid; t < L; t += NT) tw[t] = twg[t];
    const cpx<T>* src = reinterpret_cast<const cpx<T>*>(a.G) + (size_t)f * N * M * L;
    for (int t = tid; t < TILE * L; t += NT) {
        const int nn = t / L, z = t % L, n = n0 + nn;
        buf[t] = n < N ? src[((size_t)n * M + m) * L + z] : cpx<T>{T(0), T(0)};
    }
    __syncthreads();
    lds_fft<T, L, TILE, L, NT>(buf, tw, -1);
    cpx<TS>* dst = reinterpret_cast<cpx<TS>*>(a.out[f]) + (size_t)m * nk * N;
    for (int t = tid; t < nk * TILE; t += NT) {
        const int kk = t / TILE, nn = t % TILE, n = n0 + nn;
        if (n >= N) continue;
        const int k = kk - (K - 1);
        const int bin = k >= 0 ? k : L + k;
        dst[(size_t)kk * N + n] = cvt<TS>(buf[nn * L + bin]);
    }
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

template <typename TS, typename T>
static hipError_t launch_typed(const NLArgs& a, int stage, hipStream_t s) {
    const int L3K = 3 * a.K, L3M = 3 * a.M;
    const int ntile = (a.N + TILE - 1) / TILE;
    const int nzt = (L3K + TILE - 1) / TILE;
    const size_t lz = (size_t)(TILE + 1) * L3K * sizeof(cpx<T>);
    const size_t lt = (size_t)(3 * TILE + 1) * L3M * sizeof(cpx<T>);
    if (stage == 0) {
        switch (L3K) {
#define OPF_CASE(V)                                                                          \
    case V:                                                                                  \
        hipLaunchKernelGGL((k_zinv<TS, T, V>), dim3(6 * a.M * ntile), dim3(NT), lz, s, a); \
        break;
            OPF_FOR_LENGTHS(OPF_CASE)
#undef OPF_CASE
            default: return hipErrorInvalidValue;
        }
    } else if (stage == 1) {
        switch (L3M) {
#define OPF_CASE(V)                                                                \
    case V:                                                                        \
        hipLaunchKernelGGL((k_theta<T, V>), dim3(a.N * nzt), dim3(NT), lt, s, a); \
        break;
            OPF_FOR_LENGTHS(OPF_CASE)
#undef OPF_CASE
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (L3K) {
#define OPF_CASE(V)                                                                          \
    case V:                                                                                  \
        hipLaunchKernelGGL((k_zfwd<TS, T, V>), dim3(3 * a.M * ntile), dim3(NT), lz, s, a); \
        break;
            OPF_FOR_LENGTHS(OPF_CASE)
#undef OPF_CASE
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_nonlinear_stage(const NLArgs& a, int precision, int stage, hipStream_t s) {
    if (precision == OPF_MIXED) return launch_typed<float, float>(a, stage, s);
    return launch_typed<double, double>(a, stage, s);
}

hipError_t launch_nonlinear(const NLArgs& a, int precision, hipStream_t s) {
    for (int stage = 0; stage < 3; ++stage) {
        const hipError_t e = launch_nonlinear_stage(a, precision, stage, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace opf
