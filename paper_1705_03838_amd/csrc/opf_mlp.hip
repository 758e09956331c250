// Learned preconditioner of the Newton-Krylov solver: a residual MLP whose
// dense layers run on the matrix cores (bfloat16 operands, FP32
// accumulation), its backward pass and Adam; the network turns the features
// of each Fourier mode into the factors of a rank-R correction of -I, which
// k_lowrank_apply applies to the mode's radial profile, and k_head is the
// loss of that map on recorded (z, J z) pairs.
//
// Network (weights [out][in] row-major, L residual layers of width H):
//   h_0 = W_in x + b_in;  h_l = h_{l-1} + relu(W_l h_{l-1} + b_l);  y = W_out h_L + b_out.
// Every GEMM here computes C[i][j] = sum_k A[i][k] B[j][k] with both operands
// stored k-contiguous, so that each lane of a wave loads 8 consecutive
// bfloat16 values of A and of B straight into the operand registers of
// v_mfma_f32_32x32x16_bf16: the forward pass takes B = W, the input gradient
// takes B = W^T (a transposed bfloat16 copy kept beside each weight), and the
// weight gradient takes A = dZ^T, B = H^T (transposed activations written by
// the epilogues of the forward and backward GEMMs).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "opf_internal.h"

using namespace opf;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16_t;  // storage of one bfloat16 value

constexpr int NCOND = 32;  // conditioning features per row
constexpr int GT = 32;     // rows and columns of C per GEMM workgroup
constexpr int MAXL = 8;    // residual layers
constexpr int MAXSEG = 2 * MAXL + 4;

// float -> bfloat16, round to nearest, ties to even (finite inputs)
__host__ __device__ inline bf16_t f2bf(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

enum { EPI_PLAIN = 0, EPI_RELU_RES = 1, EPI_ADD = 2 };

// What the GEMM epilogue does with v = acc (+ bias[col]):
//   zout <- v;  v <- res + relu(v) (RELU_RES) or res + v (ADD);  out <- v;
//   w = v, or 0 where mask <= 0;  outb[row][col] <- bf16(w);  outT[col][row] <- bf16(w).
// Every pointer may be null (that store is skipped).
struct Epi {
    const float* bias;
    float* zout;
    int ldz;
    int mode;
    const float* res;
    int ldr;
    float* out;
    int ldo;
    const float* mask;
    int ldm;
    bf16_t* outb;
    int ldb;
    bf16_t* outT;
    int ldt;
};

__device__ __forceinline__ void epilogue(const Epi& e, int row, int col, float s) {
    float v = s + (e.bias ? e.bias[col] : 0.0f);
    if (e.zout) e.zout[(size_t)row * e.ldz + col] = v;
    if (e.mode == EPI_RELU_RES)
        v = e.res[(size_t)row * e.ldr + col] + fmaxf(v, 0.0f);
    else if (e.mode == EPI_ADD)
        v = e.res[(size_t)row * e.ldr + col] + v;
    if (e.out) e.out[(size_t)row * e.ldo + col] = v;
    float w = v;
    if (e.mask && !(e.mask[(size_t)row * e.ldm + col] > 0.0f)) w = 0.0f;
    if (e.outb) e.outb[(size_t)row * e.ldb + col] = f2bf(w);
    if (e.outT) e.outT[(size_t)col * e.ldt + row] = f2bf(w);
}

// C[rows][cols] = A[rows][K] B[cols][K]^T on v_mfma_f32_32x32x16_bf16.
// One workgroup per 32x32 tile of C; its four waves split the workgroup's
// K range [k_begin, k_end) (wave w takes the 16-wide slices w, w+4, ...) and
// their partial tiles are summed in LDS in a fixed order.  Lane l of a wave
// supplies row l%32 of the A slice and row l%32 of the B slice, elements
// 8*(l/32)..+7 (the operand layout of the instruction); accumulator entry i
// of lane l is C[8(i/4) + 4(l/32) + i%4][l%32].  The next slice's operands
// are loaded before the current product is issued.  Without a split
// (part == null) the tile goes through the epilogue; with a split over
// gridDim.z ranges of kc, workgroup z writes its raw partial tile to
// part[z][rows][cols] for k_gemm_reduce.
// Requires rows, cols multiples of 32, K and kc of 16, lda, ldb multiples of 8.
__global__ __launch_bounds__(256) void k_gemm(const bf16_t* __restrict__ A, int lda, const bf16_t* __restrict__ B,
                                              int ldb, int K, int kc, Epi e, float* __restrict__ part) {
    __shared__ float red[4][16][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int rr = lane & 31, kq = (lane >> 5) * 8;
    const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
    f32x16 acc = {};
    const bf16_t* ap = A + (size_t)(m0 + rr) * lda + kq;
    const bf16_t* bp = B + (size_t)(n0 + rr) * ldb + kq;
    int k0 = kb + wv * 16;
    u32x4 an = {}, bn = {};
    if (k0 < ke) {
        an = *reinterpret_cast<const u32x4*>(ap + k0);
        bn = *reinterpret_cast<const u32x4*>(bp + k0);
    }
    for (; k0 < ke; k0 += 64) {
        const u32x4 ac = an, bc = bn;
        if (k0 + 64 < ke) {
            an = *reinterpret_cast<const u32x4*>(ap + k0 + 64);
            bn = *reinterpret_cast<const u32x4*>(bp + k0 + 64);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ac), __builtin_bit_cast(bf16x8, bc),
                                                      acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) red[wv][i][lane] = acc[i];
    __syncthreads();
    const int cols = gridDim.x * GT, rows = gridDim.y * GT;
    for (int q = threadIdx.x; q < 1024; q += 256) {
        const int i = q >> 6, l = q & 63;
        const float s = ((red[0][i][l] + red[1][i][l]) + red[2][i][l]) + red[3][i][l];
        const int row = m0 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
        const int col = n0 + (l & 31);
        if (part)
            part[((size_t)blockIdx.z * rows + row) * cols + col] = s;
        else
            epilogue(e, row, col, s);
    }
}

// The same product for large shapes: one 128 x 128 tile of C per workgroup,
// each wave a 64 x 64 quarter (2 x 2 instruction tiles of 32 x 32, 64
// accumulators per lane).  K advances 32 at a time through double-buffered
// LDS tiles of A and B (rows padded to 40 bf16, 80 bytes, so the 16-byte
// operand reads of 16 consecutive lanes hit distinct banks); the next
// slice's global loads are issued before the current slice's products.
// Every wave takes its 64 x 64 quarter through all of K, so a C entry is the
// same K-ordered sum for every launch shape; with a split (part != null)
// workgroup z writes its raw partial tile for k_gemm_reduce.
// Requires rows, cols multiples of 128, K and kc of 32, lda, ldb of 8.
constexpr int G2 = 128, GK2 = 32, GLS2 = 40;
__global__ __launch_bounds__(256) void k_gemm128(const bf16_t* __restrict__ A, int lda,
                                                 const bf16_t* __restrict__ B, int ldb, int K, int kc, Epi e,
                                                 float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) bf16_t sa[2][G2 * GLS2];
    __shared__ __attribute__((aligned(16))) bf16_t sb[2][G2 * GLS2];
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int m0 = blockIdx.y * G2, n0 = blockIdx.x * G2;
    const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
    const int lr = t >> 2, lk = 8 * (t & 3);  // loader: rows lr and lr + 64, k lk..lk+7
    const bf16_t* ag = A + (size_t)(m0 + lr) * lda + lk;
    const bf16_t* bg = B + (size_t)(n0 + lr) * ldb + lk;
    const size_t a64 = (size_t)64 * lda, b64 = (size_t)64 * ldb;
    u32x4 ra0, ra1, rb0, rb1;
    ra0 = *reinterpret_cast<const u32x4*>(ag + kb);
    ra1 = *reinterpret_cast<const u32x4*>(ag + a64 + kb);
    rb0 = *reinterpret_cast<const u32x4*>(bg + kb);
    rb1 = *reinterpret_cast<const u32x4*>(bg + b64 + kb);
    *reinterpret_cast<u32x4*>(&sa[0][lr * GLS2 + lk]) = ra0;
    *reinterpret_cast<u32x4*>(&sa[0][(lr + 64) * GLS2 + lk]) = ra1;
    *reinterpret_cast<u32x4*>(&sb[0][lr * GLS2 + lk]) = rb0;
    *reinterpret_cast<u32x4*>(&sb[0][(lr + 64) * GLS2 + lk]) = rb1;
    __syncthreads();
    const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;
    const int rr = lane & 31, kq = (lane >> 5) * 8;
    f32x16 acc[2][2] = {};
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += GK2) {
        const bool more = k0 + GK2 < ke;
        if (more) {
            ra0 = *reinterpret_cast<const u32x4*>(ag + k0 + GK2);
            ra1 = *reinterpret_cast<const u32x4*>(ag + a64 + k0 + GK2);
            rb0 = *reinterpret_cast<const u32x4*>(bg + k0 + GK2);
            rb1 = *reinterpret_cast<const u32x4*>(bg + b64 + k0 + GK2);
        }
#pragma unroll
        for (int ks = 0; ks < GK2; ks += 16) {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = *reinterpret_cast<const bf16x8*>(&sa[buf][(wm + 32 * i + rr) * GLS2 + ks + kq]);
                bv[i] = *reinterpret_cast<const bf16x8*>(&sb[buf][(wn + 32 * i + rr) * GLS2 + ks + kq]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
            *reinterpret_cast<u32x4*>(&sa[buf ^ 1][lr * GLS2 + lk]) = ra0;
            *reinterpret_cast<u32x4*>(&sa[buf ^ 1][(lr + 64) * GLS2 + lk]) = ra1;
            *reinterpret_cast<u32x4*>(&sb[buf ^ 1][lr * GLS2 + lk]) = rb0;
            *reinterpret_cast<u32x4*>(&sb[buf ^ 1][(lr + 64) * GLS2 + lk]) = rb1;
        }
        __syncthreads();
        buf ^= 1;
    }
    const int cols = gridDim.x * G2, rows = gridDim.y * G2;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int col = n0 + wn + 32 * j + rr;
                if (part)
                    part[((size_t)blockIdx.z * rows + row) * cols + col] = acc[i][j][v];
                else
                    epilogue(e, row, col, acc[i][j][v]);
            }
}

// Sum of the split partial tiles in order, then the epilogue.
__global__ void k_gemm_reduce(const float* __restrict__ part, int rows, int cols, int nsplit, Epi e) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)rows * cols) return;
    float s = 0.0f;
    for (int z = 0; z < nsplit; ++z) s += part[(size_t)z * rows * cols + i];
    epilogue(e, (int)(i / cols), (int)(i % cols), s);
}

// FP32 rows [nrows][d] -> bfloat16 rows [rp][d] and transposed [d][ldt];
// rows nrows..rp-1 become zero.
__global__ void k_rows_bf16(const float* __restrict__ x, int nrows, int rp, int d, bf16_t* xb, bf16_t* xt,
                            int ldt) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)rp * d) return;
    const int row = (int)(i / d), col = (int)(i % d);
    const bf16_t b = f2bf(row < nrows ? x[i] : 0.0f);
    if (xb) xb[i] = b;
    if (xt) xt[(size_t)col * ldt + row] = b;
}

__device__ inline float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum of om[0..n) (or n when om is null) into *out; one workgroup.
__global__ __launch_bounds__(256) void k_weight_sum(const float* __restrict__ om, int n, float* out) {
    __shared__ float part[4];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += om ? om[i] : 1.0f;
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = ((part[0] + part[1]) + part[2]) + part[3];
}

// Weighted squared error, rows < nrows: loss_r = om_r sum_j (y - t)^2,
// dY = 2 om_r (y - t) / W with W = sum_r om_r (om null: om_r = 1).  dY
// replaces Y in place; bfloat16 copies go to dyb [rp][d] and dyt [d][ldt].
// Rows nrows..rp-1 get dY = 0.  One wave per row.
__global__ __launch_bounds__(256) void k_loss(float* __restrict__ y, const float* __restrict__ t,
                                              const float* __restrict__ om, const float* __restrict__ wsum,
                                              int nrows, int rp, int d, bf16_t* dyb, bf16_t* dyt, int ldt,
                                              float* __restrict__ lrow) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rp) return;
    const bool live = row < nrows;
    const float w = live ? (om ? om[row] : 1.0f) : 0.0f;
    const float g = 2.0f * w / *wsum;
    float acc = 0.0f;
    for (int j = lane; j < d; j += 64) {
        const size_t i = (size_t)row * d + j;
        const float r = live ? y[i] - t[i] : 0.0f;
        acc += r * r;
        const float dy = g * r;
        y[i] = dy;
        const bf16_t b = f2bf(dy);
        dyb[i] = b;
        dyt[(size_t)j * ldt + row] = b;
    }
    acc = wave_sum(acc);
    if (lane == 0) lrow[row] = w * acc;
}

// *out = sum_r lrow[r] / *wsum, rows < n; one workgroup.
__global__ __launch_bounds__(256) void k_loss_total(const float* __restrict__ lrow, int n,
                                                    const float* __restrict__ wsum, float* out) {
    __shared__ float part[4];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += lrow[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (((part[0] + part[1]) + part[2]) + part[3]) / *wsum;
}

// Column sums in two passes (bias gradients):
// part[c][col] = sum over rows c*ch .. c*ch+ch-1 (< rows) of src[row][col]
// (times [mask > 0] when mask is given), 32 columns x 8 row groups per
// workgroup; then out[col] = sum_c part[c][col] in order.  Deterministic.
constexpr int CS_CHUNKS = 64;  // largest number of row chunks
constexpr int GSPLIT = 8;                     // largest K split of a GEMM
constexpr size_t GPART = (size_t)1 << 23;     // floats of split partial tiles (split x rows x cols)
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ src, const float* __restrict__ mask,
                                                     int rows, int ld, int ch, float* __restrict__ part) {
    __shared__ float red[8][32];
    const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int col = blockIdx.x * 32 + c;
    const int r0 = blockIdx.y * ch, r1 = min(rows, r0 + ch);
    float s = 0.0f;
    for (int r = r0 + g; r < r1; r += 8) {
        const size_t i = (size_t)r * ld + col;
        const float v = src[i];
        s += (!mask || mask[i] > 0.0f) ? v : 0.0f;
    }
    red[g][c] = s;
    __syncthreads();
    if (g == 0) {
        float t = 0.0f;
        for (int q = 0; q < 8; ++q) t += red[q][c];
        part[(size_t)blockIdx.y * ld + col] = t;
    }
}
__global__ void k_colsum_fin(const float* __restrict__ part, int nch, int ld, float* __restrict__ out) {
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= ld) return;
    float t = 0.0f;
    for (int c = 0; c < nch; ++c) t += part[(size_t)c * ld + col];
    out[col] = t;
}

// Parameter segments: weight matrices [rows][cols] and bias vectors.
struct Segs {
    int n;
    long off[MAXSEG + 1];
    int rows[MAXSEG], cols[MAXSEG], mat[MAXSEG];
};

__device__ inline int seg_of(const Segs& s, long i) {
    int j = 0;
    while (j + 1 < s.n && i >= s.off[j + 1]) ++j;
    return j;
}

// bfloat16 copies of the weights: wb [rows][cols] at the parameter offset,
// wt [cols][rows] at the same offset.
__device__ inline void store_copies(const Segs& s, long i, float p, bf16_t* wb, bf16_t* wt) {
    const int j = seg_of(s, i);
    if (!s.mat[j]) return;
    const long loc = i - s.off[j];
    const int r = (int)(loc / s.cols[j]), c = (int)(loc % s.cols[j]);
    const bf16_t b = f2bf(p);
    wb[i] = b;
    wt[s.off[j] + (long)c * s.rows[j] + r] = b;
}

__global__ void k_refresh(const float* __restrict__ p, long n, Segs s, bf16_t* wb, bf16_t* wt) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    store_copies(s, i, p[i], wb, wt);
}

// Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m c1) / (sqrt(v c2) + eps), c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float c1, float c2, float eps,
                       Segs s, bf16_t* wb, bf16_t* wt) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    store_copies(s, i, pi, wb, wt);
}

}  // namespace

// ---------------------------------------------------------------------------
// The preconditioner: per-mode low-rank corrections generated by the network.
namespace {

constexpr int RMAX = 32;  // largest rank

// Conditioning features of mode (m, k): mu = mp m (azimuthal wavenumber),
// kappa = alpha k (axial wavenumber).
__device__ inline float cond_feature(int j, int mi, int k, int mp, double alpha) {
    const double mu = (double)mp * mi, ka = alpha * k;
    switch (j) {
        case 0: return 1.0f;
        case 1: return (float)(mu / 48.0);
        case 2: return (float)(ka / 40.0);
        case 3: return (float)(fabs(ka) / 40.0);
        case 4: return (float)((ka > 0) - (ka < 0));
        case 5: return (float)((mu / 48.0) * (mu / 48.0));
        case 6: return (float)((ka / 40.0) * (ka / 40.0));
        case 7: return (float)(mu * fabs(ka) / 1920.0);
        default: break;
    }
    if (j < 16) return mi == j - 8 ? 1.0f : 0.0f;
    if (j < 31) return k == j - 23 ? 1.0f : 0.0f;
    return (k > 7 || k < -7) ? 1.0f : 0.0f;
}

// One row of NCOND features per mode q = m (2K-1) + k + K-1; rows past M(2K-1)
// are zero.
__global__ void k_features(float* __restrict__ fx, int rows, int rp, int nk, int K, int mp, double alpha) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= rp * NCOND) return;
    const int q = i / NCOND, j = i % NCOND;
    fx[i] = q < rows ? cond_feature(j, q / nk, q % nk - (K - 1), mp, alpha) : 0.0f;
}

// Output row of mode q: A[e][j] at 2(e R + j) (+1 imaginary), e < 3N, j < R;
// B at the same places from offset 6 N R on.

// z_q = -v_q + A_q (B_q^H v_q) with v_q the profile of mode q (e = c N + n);
// (m = 0, k < 0) is the conjugate of (0, -k), (0, 0) keeps its real part.
// One wave per output mode; the waves of a workgroup share nothing.
__global__ __launch_bounds__(256) void k_lowrank_apply(const float* __restrict__ fac, int dout, int rank,
                                                       const double* __restrict__ v, double* __restrict__ z, int N,
                                                       int M, int nk, int K) {
    __shared__ double cs[4][2 * RMAX];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q0 = blockIdx.x * 4 + w;
    if (q0 >= M * nk) return;
    const int mi = q0 / nk, kk = q0 % nk;
    const bool mir = mi == 0 && kk < K - 1;
    const int q = mir ? 2 * (K - 1) - kk : q0;
    const long S = (long)M * nk * N;
    const int n3 = 3 * N;
    const float* A = fac + (long)q * dout;
    const float* B = A + 6 * N * rank;
    double yr[3], yi[3];
    for (int t = 0; t < 3; ++t) {
        const int e = lane + 64 * t;
        yr[t] = yi[t] = 0.0;
        if (e < n3) {
            const long idx = (e / N) * S + (long)q * N + e % N;
            yr[t] = v[2 * idx];
            yi[t] = v[2 * idx + 1];
        }
    }
    for (int j = 0; j < rank; ++j) {  // c_j = sum_e conj(B_ej) y_e
        double cr = 0.0, ci = 0.0;
        for (int t = 0; t < 3; ++t) {
            const int e = lane + 64 * t;
            if (e < n3) {
                const double br = B[2 * (e * rank + j)], bi = B[2 * (e * rank + j) + 1];
                cr += br * yr[t] + bi * yi[t];
                ci += br * yi[t] - bi * yr[t];
            }
        }
        // every lane holds the same sum and stores it: each lane reads back its own store
        cs[w][2 * j] = wave_sum(cr);
        cs[w][2 * j + 1] = wave_sum(ci);
    }
    for (int t = 0; t < 3; ++t) {
        const int e = lane + 64 * t;
        if (e >= n3) continue;
        double zr = -yr[t], zi = -yi[t];
        for (int j = 0; j < rank; ++j) {
            const double ar = A[2 * (e * rank + j)], ai = A[2 * (e * rank + j) + 1];
            const double cr = cs[w][2 * j], ci = cs[w][2 * j + 1];
            zr += ar * cr - ai * ci;
            zi += ar * ci + ai * cr;
        }
        if (mir) zi = -zi;
        if (mi == 0 && kk == K - 1) zi = 0.0;
        const long out = (e / N) * S + (long)q0 * N + e % N;
        z[2 * out] = zr;
        z[2 * out + 1] = zi;
    }
}

struct HeadArgs {
    const double* pairs;  // [npairs][2][3][M][2K-1][N] complex: (z, J z)
    long vec;             // doubles per vector
    const int* idx;       // pair indices of the batch
    int batch;
    int N, M, nk, rank, dout;
    int rows, rp;  // M(2K-1) live rows, rows padded to 32
    float* Y;      // in: network output rows; out: dLoss/dY
    bf16_t* dyb;   // [rp][dout]
    float* lrow;   // per-row loss
    float scale;   // 1 / (batch rows)
    int hb;        // pairs per pass (head_pairs)
};

constexpr int HB = 8;             // most pairs staged per pass of the loss head
constexpr int HOUT = 12;          // gradient outputs per thread and factor: 3N R <= 256 HOUT
constexpr int HEAD_LDS = 53248;   // LDS bytes of one loss-head workgroup at most (three per compute unit)

// float2 slots of the loss head's LDS for nb pairs per pass: U and V rows
// padded to R + 1 entries, the nb staged profiles xhat and that (then r),
// C and G, and 256 partial sums.
__host__ __device__ inline int head_slots(int n3, int R, int nb) {
    return 2 * n3 * (R + 1) + nb * (2 * n3 + 2 * R) + 256;
}
// Pairs per pass that fit HEAD_LDS, at least 1.  Every admissible grid
// (3N R <= 3072, 3N <= 192) needs at most 7200 slots (57.6 KB) for one pair,
// within the 64 KB a workgroup may take.
inline int head_pairs(int n3, int R) {
    int nb = HB;
    while (nb > 1 && head_slots(n3, R, nb) * 8 > HEAD_LDS) --nb;
    return nb;
}

// Loss head of the training pairs: the network's factors U = A, V = B model
// the Jacobian on each mode, J_q ~ -I + U V^H.  For mode q and pair p:
// s = RMS of the z_q profile (pairs with s = 0 skip), xhat = z_q / s,
// that = (J z)_q / s, c = V^H xhat, r = -xhat + U c - that;
// loss = scale sum |r|^2, dU = 2 scale sum r c^H, dV = 2 scale sum xhat (U^H r)^H.
// One workgroup of 256 threads per row.  The row's U and V are staged in LDS
// once (rows padded to R + 1 entries, so threads over consecutive e spread
// over the banks); pairs pass through LDS hb at a time (FP32).  Per pass:
// C = V^H X and G = U^H R with the sum over e split into np ranges whose
// partial sums are added in a fixed order, R = -X + U C - T by threads over
// (pair, e), and dU += R C^H, dV += X G^H in registers (each thread owns
// fixed gradient entries) until the row is written once: dY in FP32 and its
// row-major bfloat16 copy (k_transpose_bf16 makes the transposed one).
// HO: gradient entries per thread and factor (3N R <= 256 HO); JFIX: R
// divides 256, so every entry of a thread has the same j and the thread
// keeps C and G of its column in registers through the dU, dV update.
template <int HO, bool JFIX>
__global__ __launch_bounds__(256) void k_head(HeadArgs a) {
    extern __shared__ float2 hsm[];
    __shared__ float sinv[HB];
    __shared__ float lpart[4];
    const int q = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    float* yrow = a.Y + (long)q * a.dout;
    const int n3 = 3 * a.N, R = a.rank, RP = R + 1, nf = n3 * R;  // complex entries of U (and of V)
    if (q >= a.rows) {  // padding rows: zero gradient
        for (int j = t; j < a.dout; j += 256) {
            yrow[j] = 0.0f;
            a.dyb[(long)q * a.dout + j] = 0;
        }
        if (t == 0) a.lrow[q] = 0.0f;
        return;
    }
    const int hb = a.hb;
    float2* sU = hsm;               // [n3][RP]
    float2* sV = sU + n3 * RP;      // [n3][RP]
    float2* xs = sV + n3 * RP;      // [hb][n3]: xhat, kept for dV
    float2* rs = xs + hb * n3;      // [hb][n3]: that, then r
    float2* cs = rs + hb * n3;      // [hb][R]
    float2* gs = cs + hb * R;       // [hb][R]
    float2* red = gs + hb * R;      // [256] partial sums
    {
        const float2* U2 = reinterpret_cast<const float2*>(yrow);
        for (int i = t; i < nf; i += 256) {
            const int e = i / R, j = i - e * R;
            sU[e * RP + j] = U2[i];
            sV[e * RP + j] = U2[nf + i];
        }
    }
    const long S = (long)a.M * a.nk * a.N;
    float2 du[HO], dv[HO];
#pragma unroll
    for (int o = 0; o < HO; ++o) du[o] = dv[o] = make_float2(0.0f, 0.0f);
    float lsum = 0.0f;
    for (int b0 = 0; b0 < a.batch; b0 += hb) {
        const int nb = min(hb, a.batch - b0);
        const int items = nb * R;
        const int np = items >= 256 ? 1 : 256 / items;  // e ranges of the V^H X and U^H R sums
        const int elen = (n3 + np - 1) / np;
        for (int i = t; i < nb * n3; i += 256) {  // stage z and J z profiles of mode q
            const int b = i / n3, e = i - b * n3;
            const double* zv = a.pairs + (long)a.idx[b0 + b] * 2 * a.vec;
            const long idx = (e / a.N) * S + (long)q * a.N + e % a.N;
            const double2 zz = *reinterpret_cast<const double2*>(zv + 2 * idx);
            const double2 jz = *reinterpret_cast<const double2*>(zv + a.vec + 2 * idx);
            xs[i] = make_float2((float)zz.x, (float)zz.y);
            rs[i] = make_float2((float)jz.x, (float)jz.y);
        }
        __syncthreads();
        for (int b = w; b < nb; b += 4) {  // s of each pair: one wave per pair
            float s2 = 0.0f;
            for (int e = lane; e < n3; e += 64) s2 += xs[b * n3 + e].x * xs[b * n3 + e].x + xs[b * n3 + e].y * xs[b * n3 + e].y;
            s2 = wave_sum(s2);
            if (lane == 0) sinv[b] = s2 > 0.0f ? 1.0f / sqrtf(s2 / n3) : 0.0f;
        }
        __syncthreads();
        for (int i = t; i < nb * n3; i += 256) {
            const float f = sinv[i / n3];
            xs[i].x *= f;
            xs[i].y *= f;
            rs[i].x *= f;
            rs[i].y *= f;
        }
        __syncthreads();
        for (int i = t; i < items * np; i += 256) {  // partial C = V^H X over e range p
            const int p = i / items, bj = i - p * items, b = bj / R, j = bj - b * R;
            const int e0 = p * elen, e1 = min(n3, e0 + elen);
            float cr = 0.0f, ci = 0.0f;
#pragma unroll 4
            for (int e = e0; e < e1; ++e) {
                const float2 v = sV[e * RP + j], x = xs[b * n3 + e];
                cr += v.x * x.x + v.y * x.y;
                ci += v.x * x.y - v.y * x.x;
            }
            if (np == 1) cs[bj] = make_float2(cr, ci);
            else red[i] = make_float2(cr, ci);
        }
        __syncthreads();
        if (np > 1) {
            for (int bj = t; bj < items; bj += 256) {
                float2 c = red[bj];
                for (int p = 1; p < np; ++p) c.x += red[p * items + bj].x, c.y += red[p * items + bj].y;
                cs[bj] = c;
            }
            __syncthreads();
        }
        for (int i = t; i < nb * n3; i += 256) {  // r = -x + U c - that
            const int b = i / n3, e = i - b * n3;
            const float2 x = xs[i], th = rs[i];
            float pr = -x.x - th.x, pi = -x.y - th.y;
#pragma unroll 4
            for (int j = 0; j < R; ++j) {
                const float2 u = sU[e * RP + j], c = cs[b * R + j];
                pr += u.x * c.x - u.y * c.y;
                pi += u.x * c.y + u.y * c.x;
            }
            rs[i] = make_float2(pr, pi);
            lsum += pr * pr + pi * pi;
        }
        __syncthreads();
        for (int i = t; i < items * np; i += 256) {  // partial G = U^H R over e range p
            const int p = i / items, bj = i - p * items, b = bj / R, j = bj - b * R;
            const int e0 = p * elen, e1 = min(n3, e0 + elen);
            float gr = 0.0f, gi = 0.0f;
#pragma unroll 4
            for (int e = e0; e < e1; ++e) {
                const float2 u = sU[e * RP + j], r = rs[b * n3 + e];
                gr += u.x * r.x + u.y * r.y;
                gi += u.x * r.y - u.y * r.x;
            }
            if (np == 1) gs[bj] = make_float2(gr, gi);
            else red[i] = make_float2(gr, gi);
        }
        __syncthreads();
        if (np > 1) {
            for (int bj = t; bj < items; bj += 256) {
                float2 g = red[bj];
                for (int p = 1; p < np; ++p) g.x += red[p * items + bj].x, g.y += red[p * items + bj].y;
                gs[bj] = g;
            }
            __syncthreads();
        }
        if constexpr (JFIX) {  // dU += r c^H, dV += x g^H on this thread's entries (column j0)
            const int j0 = t % R, e0 = t / R, es = 256 / R;
#pragma unroll 2
            for (int b = 0; b < nb; ++b) {
                const float2 c = cs[b * R + j0], g = gs[b * R + j0];
#pragma unroll
                for (int o = 0; o < HO; ++o) {
                    const int e = e0 + es * o;
                    if (e < n3) {
                        const float2 r = rs[b * n3 + e], x = xs[b * n3 + e];
                        du[o].x += r.x * c.x + r.y * c.y;
                        du[o].y += r.y * c.x - r.x * c.y;
                        dv[o].x += x.x * g.x + x.y * g.y;
                        dv[o].y += x.y * g.x - x.x * g.y;
                    }
                }
            }
        } else {
#pragma unroll
            for (int o = 0; o < HO; ++o) {
                const int i = t + 256 * o;
                if (i < nf) {
                    const int e = i / R, j = i - e * R;
                    for (int b = 0; b < nb; ++b) {
                        const float2 r = rs[b * n3 + e], c = cs[b * R + j];
                        du[o].x += r.x * c.x + r.y * c.y;
                        du[o].y += r.y * c.x - r.x * c.y;
                        const float2 x = xs[b * n3 + e], g = gs[b * R + j];
                        dv[o].x += x.x * g.x + x.y * g.y;
                        dv[o].y += x.y * g.x - x.x * g.y;
                    }
                }
            }
        }
        __syncthreads();
    }
    lsum = wave_sum(lsum);
    if (lane == 0) lpart[w] = lsum;
    __syncthreads();
    if (t == 0) a.lrow[q] = ((lpart[0] + lpart[1]) + lpart[2]) + lpart[3];
    const float g2 = 2.0f * a.scale;
    float2* y2 = reinterpret_cast<float2*>(yrow);
    uint32_t* yb = reinterpret_cast<uint32_t*>(a.dyb + (long)q * a.dout);  // bf16 pairs
#pragma unroll
    for (int o = 0; o < HO; ++o) {
        const int i = t + 256 * o;  // with JFIX: e = e0 + es o, j = j0, i.e. the same i
        if (i < nf) {
            const float2 gu = make_float2(g2 * du[o].x, g2 * du[o].y), gv = make_float2(g2 * dv[o].x, g2 * dv[o].y);
            y2[i] = gu;
            y2[nf + i] = gv;
            yb[i] = (uint32_t)f2bf(gu.x) | ((uint32_t)f2bf(gu.y) << 16);
            yb[nf + i] = (uint32_t)f2bf(gv.x) | ((uint32_t)f2bf(gv.y) << 16);
        }
    }
    for (int j = 4 * nf + t; j < a.dout; j += 256) {
        yrow[j] = 0.0f;
        a.dyb[(long)q * a.dout + j] = 0;
    }
}

// dst[c][r] = src[r][c] for r < rows, c < cols (bfloat16), through a 64 x 64
// LDS tile so that both the reads and the writes are row-contiguous.
__global__ __launch_bounds__(256) void k_transpose_bf16(const bf16_t* __restrict__ src, int rows, int cols, int lds,
                                                        bf16_t* __restrict__ dst, int ldd) {
    __shared__ bf16_t tile[64][66];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int y = ty; y < 64; y += 4) {
        const int r = r0 + y, c = c0 + tx;
        tile[y][tx] = (r < rows && c < cols) ? src[(size_t)r * lds + c] : (bf16_t)0;
    }
    __syncthreads();
    for (int y = ty; y < 64; y += 4) {
        const int c = c0 + y, r = r0 + tx;
        if (c < cols && r < rows) dst[(size_t)c * ldd + r] = tile[tx][y];
    }
}

// Preconditioner factors from the Jacobian model of each mode: with
// J_q ~ -I + U V^H, J_q^{-1} = -(I + U G^{-1} V^H), G = I_R - V^H U
// (Sherman-Morrison-Woodbury), so P(v) = -v + A (B^H v) with A = -U G^{-1},
// B = V.  G is inverted by Gauss-Jordan elimination with partial pivoting in
// FP64; a mode whose G has a zero pivot gets A = 0 (P = -I there) and
// singular[q] = 1.  One workgroup of one wave per mode.
__global__ __launch_bounds__(64) void k_woodbury(const float* __restrict__ uv, float* __restrict__ fac, int dout,
                                                 int N, int rank, int rows, int* __restrict__ singular) {
    __shared__ double g[RMAX][2 * RMAX];   // G, then its inverse (complex, row-major)
    __shared__ double gi[RMAX][2 * RMAX];
    const int q = blockIdx.x, lane = threadIdx.x;
    if (q >= rows) return;
    const int R = rank, n3 = 3 * N, nf = 6 * N * R;
    const float* U = uv + (long)q * dout;
    const float* V = U + nf;
    float* A = fac + (long)q * dout;
    float* B = A + nf;
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) {  // (V^H U)_ij = sum_e conj(V_ei) U_ej
            double sr = 0.0, si = 0.0;
            for (int e = lane; e < n3; e += 64) {
                const double vr = V[2 * (e * R + i)], vi = V[2 * (e * R + i) + 1];
                const double ur = U[2 * (e * R + j)], ui = U[2 * (e * R + j) + 1];
                sr += vr * ur + vi * ui;
                si += vr * ui - vi * ur;
            }
            sr = wave_sum(sr);
            si = wave_sum(si);
            if (lane == 0) {
                g[i][2 * j] = (i == j ? 1.0 : 0.0) - sr;
                g[i][2 * j + 1] = -si;
            }
        }
    __shared__ int bad;
    if (lane == 0) {  // Gauss-Jordan on [G | I]
        bad = 0;
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j) {
                gi[i][2 * j] = i == j ? 1.0 : 0.0;
                gi[i][2 * j + 1] = 0.0;
            }
        for (int c = 0; c < R && !bad; ++c) {
            int piv = c;
            double best = -1.0;
            for (int i = c; i < R; ++i) {
                const double m = g[i][2 * c] * g[i][2 * c] + g[i][2 * c + 1] * g[i][2 * c + 1];
                if (m > best) {
                    best = m;
                    piv = i;
                }
            }
            if (!(best > 0.0)) {
                bad = 1;
                break;
            }
            for (int j = 0; j < 2 * R; ++j) {
                const double t = g[c][j];
                g[c][j] = g[piv][j];
                g[piv][j] = t;
                const double u = gi[c][j];
                gi[c][j] = gi[piv][j];
                gi[piv][j] = u;
            }
            const double pr = g[c][2 * c], pi = g[c][2 * c + 1];
            const double den = pr * pr + pi * pi;
            const double ir = pr / den, ii = -pi / den;  // 1 / pivot
            for (int j = 0; j < R; ++j) {
                double a = g[c][2 * j], b = g[c][2 * j + 1];
                g[c][2 * j] = a * ir - b * ii;
                g[c][2 * j + 1] = a * ii + b * ir;
                a = gi[c][2 * j];
                b = gi[c][2 * j + 1];
                gi[c][2 * j] = a * ir - b * ii;
                gi[c][2 * j + 1] = a * ii + b * ir;
            }
            for (int i = 0; i < R; ++i) {
                if (i == c) continue;
                const double fr = g[i][2 * c], fi = g[i][2 * c + 1];
                for (int j = 0; j < R; ++j) {
                    g[i][2 * j] -= fr * g[c][2 * j] - fi * g[c][2 * j + 1];
                    g[i][2 * j + 1] -= fr * g[c][2 * j + 1] + fi * g[c][2 * j];
                    gi[i][2 * j] -= fr * gi[c][2 * j] - fi * gi[c][2 * j + 1];
                    gi[i][2 * j + 1] -= fr * gi[c][2 * j + 1] + fi * gi[c][2 * j];
                }
            }
        }
        singular[q] = bad;
    }
    __syncthreads();
    for (int e = lane; e < n3; e += 64)
        for (int j = 0; j < R; ++j) {  // A = -U G^{-1}, B = V
            double ar = 0.0, ai = 0.0;
            if (!bad)
                for (int i = 0; i < R; ++i) {
                    const double ur = U[2 * (e * R + i)], ui = U[2 * (e * R + i) + 1];
                    ar -= ur * gi[i][2 * j] - ui * gi[i][2 * j + 1];
                    ai -= ur * gi[i][2 * j + 1] + ui * gi[i][2 * j];
                }
            A[2 * (e * R + j)] = (float)ar;
            A[2 * (e * R + j) + 1] = (float)ai;
            B[2 * (e * R + j)] = V[2 * (e * R + j)];
            B[2 * (e * R + j) + 1] = V[2 * (e * R + j) + 1];
        }
    for (int j = 2 * nf + lane; j < dout; j += 64) A[j] = 0.0f;
}

uint64_t splitmix64(uint64_t& state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t& state) { return (double)(splitmix64(state) >> 11) * (1.0 / 9007199254740992.0); }

int round32(int x) { return (x + 31) / 32 * 32; }

}  // namespace

struct opf_mlp {
    opf_ctx* ctx = nullptr;
    hipStream_t s = nullptr;
    int N = 0, M = 0, K = 0, nk = 0, mp = 1;
    double alpha = 1.0;
    int H = 0, L = 0, rank = 0, din = 0, dout = 0, R = 0, mode_rows = 0;
    long np = 0;
    Segs segs{};
    long woff[MAXL + 2] = {}, boff[MAXL + 2] = {};
    float lr = 1e-3f, lr_final = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    long t = 0;
    bool fac_ok = false;
    float *P = nullptr, *G = nullptr, *Am = nullptr, *Av = nullptr;
    bf16_t *Wb = nullptr, *Wt = nullptr;
    bf16_t *Xb = nullptr, *XT = nullptr;
    float* Hf = nullptr;
    bf16_t *Hb = nullptr, *HT = nullptr;
    float *Z = nullptr, *Y = nullptr, *dH = nullptr;
    bf16_t *dYb = nullptr, *dYT = nullptr, *dZb0 = nullptr, *dZb1 = nullptr, *dZT = nullptr;
    float *fx = nullptr, *fac = nullptr;
    int* idx = nullptr;
    int* singular = nullptr;  // [rows] modes whose Woodbury matrix is singular
    float* part = nullptr;    // [CS_CHUNKS][max(H, dout)] column-sum partials
    float* gpart = nullptr;   // [GPART] split-K partial tiles
    int n_singular = 0;
    float *lrow = nullptr, *wsum = nullptr, *losses = nullptr;
    int loss_cap = 0;
    std::string err;

    float* hf(int l) const { return Hf + (size_t)l * R * H; }
    bf16_t* hb(int l) const { return Hb + (size_t)l * R * H; }
    bf16_t* ht(int l) const { return HT + (size_t)l * H * R; }
    float* z(int l) const { return Z + (size_t)l * R * H; }
};

namespace {

constexpr int LOSS_CAP = 1 << 16;  // training steps per call
constexpr int IDX_CAP = 1 << 20;   // pair indices per call (steps x batch)

#define MCHK(net, call)                                                             \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            (net)->err = std::string(#call) + ": " + hipGetErrorString(e_);         \
            return OPF_E_HIP;                                                       \
        }                                                                           \
    } while (0)

struct Layout {
    size_t off[32] = {};
    size_t total = 0;
    int n = 0;
    size_t take(size_t bytes) {
        const size_t o = total;
        off[n++] = o;
        total += (bytes + 255) / 256 * 256;
        return o;
    }
};

// dims, parameter segments and buffer layout of a network
Layout plan(opf_mlp* m) {
    m->din = NCOND;
    m->dout = round32(12 * m->N * m->rank);
    long o = 0;
    int j = 0;
    auto seg = [&](int rows, int cols, int mat) {
        m->segs.off[j] = o;
        m->segs.rows[j] = rows;
        m->segs.cols[j] = cols;
        m->segs.mat[j] = mat;
        ++j;
        const long at = o;
        o += (long)rows * cols;
        return at;
    };
    m->woff[0] = seg(m->H, m->din, 1);
    m->boff[0] = seg(1, m->H, 0);
    for (int l = 0; l < m->L; ++l) {
        m->woff[l + 1] = seg(m->H, m->H, 1);
        m->boff[l + 1] = seg(1, m->H, 0);
    }
    m->woff[m->L + 1] = seg(m->dout, m->H, 1);
    m->boff[m->L + 1] = seg(1, m->dout, 0);
    m->segs.n = j;
    m->segs.off[j] = o;
    m->np = o;
    const size_t R = m->R, H = m->H, L = m->L, np = o;
    Layout lay;
    for (int q = 0; q < 4; ++q) lay.take(np * 4);  // P, G, Am, Av
    lay.take(np * 2);                              // Wb
    lay.take(np * 2);                              // Wt
    lay.take(R * m->din * 2);                      // Xb
    lay.take(R * m->din * 2);                      // XT
    lay.take((L + 1) * R * H * 4);                 // Hf
    lay.take((L + 1) * R * H * 2);                 // Hb
    lay.take((L + 1) * R * H * 2);                 // HT
    lay.take(L * R * H * 4);                       // Z
    lay.take(R * m->dout * 4);                     // Y
    lay.take(R * H * 4);                           // dH
    lay.take(R * m->dout * 2);                     // dYb
    lay.take(R * m->dout * 2);                     // dYT
    lay.take(R * H * 2);                           // dZb0
    lay.take(R * H * 2);                           // dZb1
    lay.take(R * H * 2);                           // dZT
    lay.take(R * m->din * 4);                      // fx: mode feature rows
    lay.take(R * m->dout * 4);                     // fac: factor rows in use
    lay.take((size_t)IDX_CAP * 4);                 // idx: pair indices
    lay.take(R * 4);                               // singular: per-mode flag of a singular G
    lay.take((size_t)CS_CHUNKS * std::max(m->H, m->dout) * 4);  // part
    lay.take(GPART * 4);                                         // gpart
    lay.take(R * 4);                               // lrow
    lay.take(256);                                 // wsum
    lay.take((size_t)LOSS_CAP * 4);                // losses
    return lay;
}

opf_status check_cfg(const opf_ctx* c, const opf_mlp_config* cfg, std::string* why) {
    if (!c || !cfg) return OPF_E_INVALID;
    const opf_params& p = ctx_params(c);
    auto bad = [&](const char* s) {
        if (why) *why = s;
        return OPF_E_INVALID;
    };
    if (cfg->width < 32 || cfg->width > 512 || cfg->width % 32) return bad("width must be a multiple of 32 in [32, 512]");
    if (cfg->layers < 1 || cfg->layers > MAXL) return bad("layers must be in [1, 8]");
    if (cfg->rank < 1 || cfg->rank > RMAX) return bad("rank must be in [1, 32]");
    if (3L * p.N * cfg->rank > 256L * HOUT) return bad("3 N rank must not exceed 3072");
    if (cfg->max_rows < 0 || cfg->max_rows > (1 << 20)) return bad("max_rows must be in [0, 2^20]");
    if (!(cfg->lr >= 0.0f) || !(cfg->lr_final >= 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->adam_eps > 0.0f))
        return bad("bad Adam parameters");
    return OPF_OK;
}

// Column sums of rows x cols FP32 src (row stride = cols) into out.
hipError_t colsum(opf_mlp* m, const float* src, const float* mask, int rows, int cols, float* out) {
    const int ch = std::max(128, (rows + CS_CHUNKS - 1) / CS_CHUNKS);
    const int nch = (rows + ch - 1) / ch;
    hipLaunchKernelGGL(k_colsum_part, dim3(cols / 32, nch), dim3(256), 0, m->s, src, mask, rows, cols, ch, m->part);
    hipLaunchKernelGGL(k_colsum_fin, dim3((cols + 255) / 256), dim3(256), 0, m->s, m->part, nch, cols, out);
    return hipGetLastError();
}

// Launch a GEMM; one whose tile count cannot fill the chip but whose K is
// long is split over K (partial tiles to the scratch, then k_gemm_reduce).
hipError_t gemm(opf_mlp* m, const bf16_t* A, int lda, const bf16_t* B, int ldb, int rows, int cols, int K,
                const Epi& e) {
    if (rows % GT || cols % GT || K % 16 || lda % 8 || ldb % 8 || rows <= 0 || cols <= 0 || K <= 0)
        return hipErrorInvalidValue;
    if (rows % G2 == 0 && cols % G2 == 0 && K % GK2 == 0 && (double)rows * cols * K >= (double)(1L << 30)) {
        // large product: 128 x 128 tiles, K split until about 256 workgroups
        const long tiles = (long)(rows / G2) * (cols / G2);
        int nsplit = 1, kc = K;
        if (tiles < 256) {
            nsplit = (int)std::min<long>((256 + tiles - 1) / tiles, std::min(K / 256, 2 * GSPLIT));
            if ((size_t)nsplit * rows * cols > GPART) nsplit = (int)(GPART / ((size_t)rows * cols));
            nsplit = std::max(nsplit, 1);
            kc = (K + nsplit - 1) / nsplit;
            kc = (kc + GK2 - 1) / GK2 * GK2;
            nsplit = (K + kc - 1) / kc;
        }
        if (nsplit == 1) {
            hipLaunchKernelGGL(k_gemm128, dim3(cols / G2, rows / G2, 1), dim3(256), 0, m->s, A, lda, B, ldb, K, K, e,
                               nullptr);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_gemm128, dim3(cols / G2, rows / G2, nsplit), dim3(256), 0, m->s, A, lda, B, ldb, K, kc,
                           e, m->gpart);
        const size_t n = (size_t)rows * cols;
        hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->s, m->gpart, rows,
                           cols, nsplit, e);
        return hipGetLastError();
    }
    const long tiles = (long)(rows / GT) * (cols / GT);
    int nsplit = 1, kc = K;
    if (tiles < 1024 && K >= 512) {
        nsplit = (int)std::min<long>((2048 + tiles - 1) / tiles, std::min(K / 256, GSPLIT));
        kc = (K + nsplit - 1) / nsplit;
        kc = (kc + 63) / 64 * 64;
        nsplit = (K + kc - 1) / kc;
        if ((size_t)nsplit * rows * cols > GPART) nsplit = 1, kc = K;
    }
    if (nsplit == 1) {
        hipLaunchKernelGGL(k_gemm, dim3(cols / GT, rows / GT, 1), dim3(256), 0, m->s, A, lda, B, ldb, K, K, e,
                           nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_gemm, dim3(cols / GT, rows / GT, nsplit), dim3(256), 0, m->s, A, lda, B, ldb, K, kc, e,
                       m->gpart);
    const size_t n = (size_t)rows * cols;
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->s, m->gpart, rows, cols,
                       nsplit, e);
    return hipGetLastError();
}

// Forward pass over rp rows (multiple of 32) of bfloat16 rows Xb.
// train: also keep pre-activations and transposed activations.
hipError_t forward(opf_mlp* m, int rp, bool train) {
    const int H = m->H, L = m->L;
    Epi e{};
    e.bias = m->P + m->boff[0];
    e.out = m->hf(0);
    e.ldo = H;
    e.outb = m->hb(0);
    e.ldb = H;
    if (train) {
        e.outT = m->ht(0);
        e.ldt = m->R;
    }
    hipError_t st = gemm(m, m->Xb, m->din, m->Wb + m->woff[0], m->din, rp, H, m->din, e);
    if (st != hipSuccess) return st;
    for (int l = 0; l < L; ++l) {
        Epi f{};
        f.bias = m->P + m->boff[l + 1];
        if (train) {
            f.zout = m->z(l);
            f.ldz = H;
            f.outT = m->ht(l + 1);
            f.ldt = m->R;
        }
        f.mode = EPI_RELU_RES;
        f.res = m->hf(l);
        f.ldr = H;
        f.out = m->hf(l + 1);
        f.ldo = H;
        f.outb = m->hb(l + 1);
        f.ldb = H;
        st = gemm(m, m->hb(l), H, m->Wb + m->woff[l + 1], H, rp, H, H, f);
        if (st != hipSuccess) return st;
    }
    Epi g{};
    g.bias = m->P + m->boff[L + 1];
    g.out = m->Y;
    g.ldo = m->dout;
    return gemm(m, m->hb(L), H, m->Wb + m->woff[L + 1], H, rp, m->dout, H, g);
}

// Parameter gradients from dL/dY (FP32 in Y, bfloat16 in dYb / dYT) after
// forward(train = true) over rp rows.
hipError_t backprop(opf_mlp* m, int rp) {
    const int H = m->H, L = m->L, R = m->R, dout = m->dout;
    hipError_t st;
    {  // output layer: dW = dY^T H_L, db = colsum dY, dH_L = dY W_out
        Epi e{};
        e.out = m->G + m->woff[L + 1];
        e.ldo = H;
        if ((st = gemm(m, m->dYT, R, m->ht(L), R, dout, H, rp, e)) != hipSuccess) return st;
        if ((st = colsum(m, m->Y, nullptr, rp, dout, m->G + m->boff[L + 1])) != hipSuccess) return st;
        Epi f{};
        f.out = m->dH;
        f.ldo = H;
        f.mask = m->z(L - 1);
        f.ldm = H;
        f.outb = m->dZb0;
        f.ldb = H;
        f.outT = m->dZT;
        f.ldt = R;
        if ((st = gemm(m, m->dYb, dout, m->Wt + m->woff[L + 1], dout, rp, H, dout, f)) != hipSuccess)
            return st;
    }
    bf16_t* dz[2] = {m->dZb0, m->dZb1};
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        // dz_l = dH_{l+1} [z_l > 0] is in dz[cur] (row-major) and dZT (transposed)
        if ((st = colsum(m, m->dH, m->z(l), rp, H, m->G + m->boff[l + 1])) != hipSuccess) return st;
        Epi e{};
        e.out = m->G + m->woff[l + 1];
        e.ldo = H;
        if ((st = gemm(m, m->dZT, R, m->ht(l), R, H, H, rp, e)) != hipSuccess) return st;
        Epi f{};
        f.mode = EPI_ADD;
        f.res = m->dH;
        f.ldr = H;
        f.out = m->dH;
        f.ldo = H;
        f.outT = m->dZT;
        f.ldt = R;
        if (l > 0) {
            f.mask = m->z(l - 1);
            f.ldm = H;
            f.outb = dz[cur ^ 1];
            f.ldb = H;
        }
        if ((st = gemm(m, dz[cur], H, m->Wt + m->woff[l + 1], H, rp, H, H, f)) != hipSuccess) return st;
        cur ^= 1;
    }
    // input layer: dW_in = dH_0^T X, db_in = colsum dH_0
    if ((st = colsum(m, m->dH, nullptr, rp, H, m->G + m->boff[0])) != hipSuccess) return st;
    Epi e{};
    e.out = m->G + m->woff[0];
    e.ldo = m->din;
    if ((st = gemm(m, m->dZT, R, m->XT, R, H, m->din, rp, e)) != hipSuccess) return st;
    return hipGetLastError();
}

// Squared-error loss of rows (targets t, weights om) into *loss_slot and
// dL/dY, then the parameter gradients.
hipError_t backward_rows(opf_mlp* m, const float* t, const float* om, int nrows, int rp, float* loss_slot) {
    hipStream_t s = m->s;
    hipLaunchKernelGGL(k_weight_sum, dim3(1), dim3(256), 0, s, om, nrows, m->wsum);
    hipLaunchKernelGGL(k_loss, dim3(rp / 4), dim3(256), 0, s, m->Y, t, om, m->wsum, nrows, rp, m->dout, m->dYb,
                       m->dYT, m->R, m->lrow);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, m->lrow, nrows, m->wsum, loss_slot);
    const hipError_t st = hipGetLastError();
    return st != hipSuccess ? st : backprop(m, rp);
}

// Loss head over pairs idx[0..batch) into *loss_slot and dL/dY, then the
// parameter gradients (forward over the mode feature rows first).
hipError_t backward_pairs(opf_mlp* m, const double* pairs, const int* idx, int batch, float* loss_slot) {
    hipStream_t s = m->s;
    const int rp = round32(m->mode_rows);
    HeadArgs a{};
    a.pairs = pairs;
    a.vec = 2L * 3 * m->M * m->nk * m->N;
    a.idx = idx;
    a.batch = batch;
    a.N = m->N;
    a.M = m->M;
    a.nk = m->nk;
    a.rank = m->rank;
    a.dout = m->dout;
    a.rows = m->mode_rows;
    a.rp = rp;
    a.Y = m->Y;
    a.dyb = m->dYb;
    a.lrow = m->lrow;
    a.scale = (float)(1.0 / ((double)batch * m->mode_rows));
    a.hb = head_pairs(3 * m->N, m->rank);
    const size_t hl = (size_t)head_slots(3 * m->N, m->rank, a.hb) * sizeof(float2);
    const int nf = 3 * m->N * m->rank, ho = nf <= 768 ? 3 : nf <= 1536 ? 6 : nf <= 2304 ? 9 : 12;
    const bool jfix = 256 % m->rank == 0;
    auto kh = jfix ? (ho == 3 ? k_head<3, true> : ho == 6 ? k_head<6, true> : ho == 9 ? k_head<9, true> : k_head<12, true>)
                   : (ho == 3 ? k_head<3, false> : ho == 6 ? k_head<6, false> : ho == 9 ? k_head<9, false> : k_head<12, false>);
    hipLaunchKernelGGL(kh, dim3(rp), dim3(256), hl, s, a);
    hipLaunchKernelGGL(k_transpose_bf16, dim3((m->dout + 63) / 64, (rp + 63) / 64), dim3(256), 0, s, m->dYb, rp,
                       m->dout, m->dout, m->dYT, m->R);
    hipLaunchKernelGGL(k_weight_sum, dim3(1), dim3(256), 0, s, nullptr, batch * m->mode_rows, m->wsum);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, m->lrow, m->mode_rows, m->wsum, loss_slot);
    const hipError_t st = hipGetLastError();
    return st != hipSuccess ? st : backprop(m, rp);
}

hipError_t adam(opf_mlp* m, float lr) {
    m->t += 1;
    m->fac_ok = false;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)m->b1, (double)m->t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)m->b2, (double)m->t)));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((m->np + 255) / 256)), dim3(256), 0, m->s, m->P, m->G, m->Am, m->Av,
                       m->np, lr, m->b1, m->b2, c1, c2, m->eps, m->segs, m->Wb, m->Wt);
    return hipGetLastError();
}

hipError_t rows_bf16(opf_mlp* m, const float* x, int nrows, int rp, bool transposed) {
    const size_t n = (size_t)rp * m->din;
    hipLaunchKernelGGL(k_rows_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->s, x, nrows, rp, m->din,
                       m->Xb, transposed ? m->XT : nullptr, m->R);
    return hipGetLastError();
}

// The mode feature rows as GEMM input (and transposed, for training).
hipError_t feature_input(opf_mlp* m) { return rows_bf16(m, m->fx, m->mode_rows, round32(m->mode_rows), true); }

// Preconditioner factors (A, B) of the current parameters into fac: the
// network's Jacobian model (U, V) per mode, inverted by Woodbury.
hipError_t refresh_factors(opf_mlp* m) {
    if (m->fac_ok) return hipSuccess;
    const int rp = round32(m->mode_rows);
    hipError_t st = feature_input(m);
    if (st == hipSuccess) st = forward(m, rp, false);
    if (st != hipSuccess) return st;
    hipLaunchKernelGGL(k_woodbury, dim3(m->mode_rows), dim3(64), 0, m->s, m->Y, m->fac, m->dout, m->N, m->rank,
                       m->mode_rows, m->singular);
    if ((st = hipGetLastError()) != hipSuccess) return st;
    std::vector<int> flags(m->mode_rows);
    if ((st = hipMemcpyAsync(flags.data(), m->singular, flags.size() * sizeof(int), hipMemcpyDeviceToHost, m->s)) !=
            hipSuccess ||
        (st = hipStreamSynchronize(m->s)) != hipSuccess)
        return st;
    m->n_singular = 0;
    for (int f : flags) m->n_singular += f;
    m->fac_ok = true;
    return hipSuccess;
}

bool same_grid(const opf_mlp* m, const opf_ctx* c) {
    const opf_params& p = ctx_params(c);
    return p.N == m->N && p.M == m->M && p.K == m->K && p.mp == m->mp && p.alpha == m->alpha;
}

}  // namespace

extern "C" {

opf_status opf_mlp_default_config(opf_mlp_config* cfg) {
    if (!cfg) return OPF_E_INVALID;
    *cfg = opf_mlp_config{};
    cfg->width = 256;
    cfg->layers = 4;
    cfg->rank = 8;
    cfg->max_rows = 0;
    cfg->seed = 1;
    cfg->lr = 1e-3f;
    cfg->beta1 = 0.9f;
    cfg->beta2 = 0.999f;
    cfg->adam_eps = 1e-8f;
    cfg->lr_final = 1e-3f;
    return OPF_OK;
}

static void dims_for(opf_mlp* m, const opf_ctx* ctx, const opf_mlp_config* cfg) {
    const opf_params& p = ctx_params(ctx);
    m->N = p.N;
    m->M = p.M;
    m->K = p.K;
    m->nk = 2 * p.K - 1;
    m->mp = p.mp;
    m->alpha = p.alpha;
    m->H = cfg->width;
    m->L = cfg->layers;
    m->rank = cfg->rank;
    m->mode_rows = p.M * m->nk;
    m->R = round32(std::max(cfg->max_rows, m->mode_rows));
}

opf_status opf_mlp_workspace_size(const opf_ctx* ctx, const opf_mlp_config* cfg, size_t* bytes) {
    if (!bytes) return OPF_E_INVALID;
    const opf_status st = check_cfg(ctx, cfg, nullptr);
    if (st != OPF_OK) return st;
    opf_mlp m;
    dims_for(&m, ctx, cfg);
    *bytes = plan(&m).total;
    return OPF_OK;
}

opf_status opf_mlp_create(opf_ctx* ctx, const opf_mlp_config* cfg, void* dev_workspace, size_t bytes,
                          opf_mlp** out) {
    if (!out || !dev_workspace) return OPF_E_INVALID;
    *out = nullptr;
    std::string why;
    opf_status st = check_cfg(ctx, cfg, &why);
    if (st != OPF_OK) {
        if (ctx) ctx_set_error(ctx, why);
        return st;
    }
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256) return OPF_E_INVALID;
    opf_mlp* m = new (std::nothrow) opf_mlp;
    if (!m) return OPF_E_NOMEM;
    m->ctx = ctx;
    m->s = ctx_stream(ctx);
    dims_for(m, ctx, cfg);
    m->lr = cfg->lr;
    m->lr_final = cfg->lr_final;
    m->b1 = cfg->beta1;
    m->b2 = cfg->beta2;
    m->eps = cfg->adam_eps;
    const Layout lay = plan(m);
    if (bytes < lay.total) {
        delete m;
        return OPF_E_NOMEM;
    }
    unsigned char* b = static_cast<unsigned char*>(dev_workspace);
    int q = 0;
    auto at = [&](auto*& ptr) { ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(b + lay.off[q++]); };
    at(m->P);
    at(m->G);
    at(m->Am);
    at(m->Av);
    at(m->Wb);
    at(m->Wt);
    at(m->Xb);
    at(m->XT);
    at(m->Hf);
    at(m->Hb);
    at(m->HT);
    at(m->Z);
    at(m->Y);
    at(m->dH);
    at(m->dYb);
    at(m->dYT);
    at(m->dZb0);
    at(m->dZb1);
    at(m->dZT);
    at(m->fx);
    at(m->fac);
    at(m->idx);
    at(m->singular);
    at(m->part);
    at(m->gpart);
    at(m->lrow);
    at(m->wsum);
    at(m->losses);
    m->loss_cap = LOSS_CAP;
    const int rp = round32(m->mode_rows);
    hipLaunchKernelGGL(k_features, dim3((rp * NCOND + 255) / 256), dim3(256), 0, m->s, m->fx, m->mode_rows, rp, m->nk,
                       m->K, m->mp, m->alpha);
    if (hipGetLastError() != hipSuccess) {
        delete m;
        return OPF_E_HIP;
    }
    // initial weights: W ~ U(-a, a), a = 1/sqrt(fan_in) (output layer 0.01 a),
    // biases 0, from SplitMix64 (Steele, Lea & Flood 2014)
    std::vector<float> host(m->np, 0.0f);
    uint64_t state = cfg->seed;
    for (int j = 0; j < m->segs.n; ++j) {
        if (!m->segs.mat[j]) continue;
        const double a = (j == m->segs.n - 2 ? 0.01 : 1.0) / std::sqrt((double)m->segs.cols[j]);
        for (long i = m->segs.off[j]; i < m->segs.off[j + 1]; ++i) host[i] = (float)(a * (2.0 * uniform01(state) - 1.0));
    }
    st = opf_mlp_set_params(m, host.data(), m->np);
    if (st != OPF_OK) {
        ctx_set_error(ctx, m->err);
        delete m;
        return st;
    }
    *out = m;
    return OPF_OK;
}

opf_status opf_mlp_destroy(opf_mlp* net) {
    delete net;
    return OPF_OK;
}

opf_status opf_mlp_dims(const opf_mlp* net, int32_t* din, int32_t* dout, int64_t* n_params) {
    if (!net) return OPF_E_INVALID;
    if (din) *din = net->din;
    if (dout) *dout = net->dout;
    if (n_params) *n_params = net->np;
    return OPF_OK;
}

opf_status opf_mlp_set_params(opf_mlp* net, const float* host, int64_t n) {
    if (!net || !host || n != net->np) return OPF_E_INVALID;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return OPF_E_INVALID;
    MCHK(net, hipMemcpyAsync(net->P, host, (size_t)n * 4, hipMemcpyHostToDevice, net->s));
    MCHK(net, hipMemsetAsync(net->Am, 0, (size_t)n * 4, net->s));
    MCHK(net, hipMemsetAsync(net->Av, 0, (size_t)n * 4, net->s));
    hipLaunchKernelGGL(k_refresh, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, net->s, net->P, (long)n, net->segs,
                       net->Wb, net->Wt);
    MCHK(net, hipGetLastError());
    MCHK(net, hipStreamSynchronize(net->s));
    net->t = 0;
    net->fac_ok = false;
    return OPF_OK;
}

opf_status opf_mlp_get_params(opf_mlp* net, float* host, int64_t n) {
    if (!net || !host || n != net->np) return OPF_E_INVALID;
    MCHK(net, hipMemcpyAsync(host, net->P, (size_t)n * 4, hipMemcpyDeviceToHost, net->s));
    MCHK(net, hipStreamSynchronize(net->s));
    return OPF_OK;
}

opf_status opf_mlp_forward(opf_mlp* net, const float* x_dev, int32_t rows, float* y_dev) {
    if (!net || !x_dev || !y_dev || rows < 1 || rows > net->R) return OPF_E_INVALID;
    const int rp = round32(rows);
    MCHK(net, rows_bf16(net, x_dev, rows, rp, false));
    MCHK(net, forward(net, rp, false));
    MCHK(net, hipMemcpyAsync(y_dev, net->Y, (size_t)rows * net->dout * 4, hipMemcpyDeviceToDevice, net->s));
    return OPF_OK;
}

opf_status opf_mlp_gradient(opf_mlp* net, const float* x_dev, const float* t_dev, const float* w_dev, int32_t rows,
                            double* loss_host, float* grad_host) {
    if (!net || !x_dev || !t_dev || rows < 1 || rows > net->R) return OPF_E_INVALID;
    const int rp = round32(rows);
    MCHK(net, rows_bf16(net, x_dev, rows, rp, true));
    MCHK(net, forward(net, rp, true));
    MCHK(net, backward_rows(net, t_dev, w_dev, rows, rp, net->losses));
    float l = 0.0f;
    MCHK(net, hipMemcpyAsync(&l, net->losses, 4, hipMemcpyDeviceToHost, net->s));
    if (grad_host) MCHK(net, hipMemcpyAsync(grad_host, net->G, (size_t)net->np * 4, hipMemcpyDeviceToHost, net->s));
    MCHK(net, hipStreamSynchronize(net->s));
    if (loss_host) *loss_host = l;
    return std::isfinite(l) ? OPF_OK : OPF_E_NUMERIC;
}

opf_status opf_mlp_train(opf_mlp* net, const float* x_dev, const float* t_dev, const float* w_dev, int32_t rows,
                         int32_t batch, int32_t epochs, uint64_t shuffle_seed, float* loss_host) {
    if (!net || !x_dev || !t_dev || rows < 1 || batch < 1 || batch > net->R || epochs < 0) return OPF_E_INVALID;
    const int nb = (rows + batch - 1) / batch;
    if ((long)nb * epochs > net->loss_cap) return OPF_E_INVALID;
    std::vector<int> order(nb);
    uint64_t state = shuffle_seed;
    int step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = 0; i < nb; ++i) order[i] = i;
        for (int i = nb - 1; i > 0; --i) std::swap(order[i], order[(int)(uniform01(state) * (i + 1))]);
        for (int i = 0; i < nb; ++i) {
            const int r0 = order[i] * batch;
            const int n = std::min(batch, rows - r0);
            const int rp = round32(n);
            MCHK(net, rows_bf16(net, x_dev + (size_t)r0 * net->din, n, rp, true));
            MCHK(net, forward(net, rp, true));
            MCHK(net, backward_rows(net, t_dev + (size_t)r0 * net->dout, w_dev ? w_dev + r0 : nullptr, n, rp,
                                    net->losses + step));
            MCHK(net, adam(net, net->lr));
            ++step;
        }
    }
    std::vector<float> l(step);
    if (step) MCHK(net, hipMemcpyAsync(l.data(), net->losses, (size_t)step * 4, hipMemcpyDeviceToHost, net->s));
    MCHK(net, hipStreamSynchronize(net->s));
    if (loss_host)
        for (int ep = 0; ep < epochs; ++ep) {
            double a = 0.0;
            for (int i = 0; i < nb; ++i) a += l[(size_t)ep * nb + i];
            loss_host[ep] = (float)(a / nb);
        }
    return OPF_OK;
}

opf_status opf_mlp_pair_gradient(opf_ctx* ctx, opf_mlp* net, const void* pairs_dev, int32_t npairs,
                                 const int32_t* idx_host, int32_t batch, double* loss_host, float* grad_host) {
    if (!ctx || !net || !pairs_dev || !idx_host || npairs < 1 || batch < 1 || batch > IDX_CAP) return OPF_E_INVALID;
    if (!same_grid(net, ctx)) return OPF_E_INVALID;
    for (int b = 0; b < batch; ++b)
        if (idx_host[b] < 0 || idx_host[b] >= npairs) return OPF_E_INVALID;
    MCHK(net, hipMemcpyAsync(net->idx, idx_host, (size_t)batch * 4, hipMemcpyHostToDevice, net->s));
    MCHK(net, feature_input(net));
    MCHK(net, forward(net, round32(net->mode_rows), true));
    MCHK(net, backward_pairs(net, static_cast<const double*>(pairs_dev), net->idx, batch, net->losses));
    float l = 0.0f;
    MCHK(net, hipMemcpyAsync(&l, net->losses, 4, hipMemcpyDeviceToHost, net->s));
    if (grad_host) MCHK(net, hipMemcpyAsync(grad_host, net->G, (size_t)net->np * 4, hipMemcpyDeviceToHost, net->s));
    MCHK(net, hipStreamSynchronize(net->s));
    if (loss_host) *loss_host = l;
    return std::isfinite(l) ? OPF_OK : OPF_E_NUMERIC;
}

opf_status opf_mlp_train_pairs(opf_ctx* ctx, opf_mlp* net, const void* pairs_dev, int32_t npairs, int32_t batch,
                               int32_t steps, uint64_t seed, float* loss_host) {
    if (!ctx || !net || !pairs_dev || npairs < 1 || batch < 1 || steps < 0) return OPF_E_INVALID;
    if ((long)batch * steps > IDX_CAP || steps > net->loss_cap) return OPF_E_INVALID;
    if (!same_grid(net, ctx)) return OPF_E_INVALID;
    // pair indices of every step: consecutive batches of per-epoch shuffles
    std::vector<int> idx((size_t)batch * steps);
    std::vector<int> perm(npairs);
    uint64_t state = seed;
    size_t filled = 0;
    while (filled < idx.size()) {
        for (int i = 0; i < npairs; ++i) perm[i] = i;
        for (int i = npairs - 1; i > 0; --i) std::swap(perm[i], perm[(int)(uniform01(state) * (i + 1))]);
        for (int i = 0; i < npairs && filled < idx.size(); ++i) idx[filled++] = perm[i];
    }
    if (!idx.empty()) MCHK(net, hipMemcpyAsync(net->idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, net->s));
    MCHK(net, feature_input(net));
    const int rp = round32(net->mode_rows);
    for (int st = 0; st < steps; ++st) {
        // cosine schedule from lr to lr_final over the call's steps
        const double c = 0.5 * (1.0 + std::cos(M_PI * st / std::max(steps, 1)));
        const float lr = (float)(net->lr_final + (net->lr - net->lr_final) * c);
        MCHK(net, forward(net, rp, true));
        MCHK(net, backward_pairs(net, static_cast<const double*>(pairs_dev), net->idx + (size_t)st * batch, batch,
                                 net->losses + st));
        MCHK(net, adam(net, lr));
    }
    if (loss_host && steps > 0) MCHK(net, hipMemcpyAsync(loss_host, net->losses, (size_t)steps * 4,
                                                         hipMemcpyDeviceToHost, net->s));
    MCHK(net, hipStreamSynchronize(net->s));  // the host index array lives until here
    return OPF_OK;
}

opf_status opf_precondition(opf_ctx* ctx, opf_mlp* net, const void* v_dev, void* z_dev) {
    if (!ctx || !net || !v_dev || !z_dev) return OPF_E_INVALID;
    if (!same_grid(net, ctx)) return OPF_E_INVALID;
    MCHK(net, refresh_factors(net));
    hipLaunchKernelGGL(k_lowrank_apply, dim3((net->mode_rows + 3) / 4), dim3(256), 0, net->s, net->fac, net->dout,
                       net->rank, static_cast<const double*>(v_dev), static_cast<double*>(z_dev), net->N, net->M,
                       net->nk, net->K);
    MCHK(net, hipGetLastError());
    return OPF_OK;
}

opf_status opf_mlp_factors(opf_mlp* net, float* host, int64_t n, int32_t* singular_modes) {
    if (!net || (host && n != (int64_t)net->mode_rows * net->dout)) return OPF_E_INVALID;
    MCHK(net, refresh_factors(net));
    if (host) MCHK(net, hipMemcpyAsync(host, net->fac, (size_t)n * 4, hipMemcpyDeviceToHost, net->s));
    MCHK(net, hipStreamSynchronize(net->s));
    if (singular_modes) *singular_modes = net->n_singular;
    return OPF_OK;
}

const char* opf_mlp_last_error(const opf_mlp* net) { return net ? net->err.c_str() : "null network"; }

}  // extern "C"
