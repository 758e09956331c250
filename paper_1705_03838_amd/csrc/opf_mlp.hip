// Learned preconditioner of the Newton-Krylov solver: a residual MLP whose
// dense layers run on the matrix cores (bfloat16 operands, FP32
// accumulation), its backward pass, Adam, and the packing of Fourier-mode
// radial profiles into network rows and back.
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

__device__ inline uint32_t pack2(float a, float b) { return (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16); }

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

// C[rows][cols] = A[rows][K] B[cols][K]^T on v_mfma_f32_32x32x16_bf16.
// One workgroup per 32x32 tile of C; its four waves split K (wave w takes
// the 16-wide slices w, w+4, ...) and their partial tiles are summed in LDS
// in a fixed order.  Lane l of a wave supplies row l%32 of the A slice and
// row l%32 of the B slice, elements 8*(l/32)..+7 (the operand layout of the
// instruction); accumulator entry i of lane l is C[8(i/4) + 4(l/32) + i%4][l%32].
// Requires rows, cols multiples of 32, K of 16, lda, ldb multiples of 8.
template <bool AF32>
__global__ __launch_bounds__(256) void k_gemm(const void* __restrict__ A, int lda, const bf16_t* __restrict__ B,
                                              int ldb, int K, Epi e) {
    __shared__ float red[4][16][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int rr = lane & 31, kq = (lane >> 5) * 8;
    f32x16 acc = {};
    const bf16_t* bp = B + (size_t)(n0 + rr) * ldb + kq;
    for (int k0 = wv * 16; k0 < K; k0 += 64) {
        bf16x8 a;
        if constexpr (AF32) {
            const float* ap = static_cast<const float*>(A) + (size_t)(m0 + rr) * lda + kq + k0;
            const float4 x0 = *reinterpret_cast<const float4*>(ap);
            const float4 x1 = *reinterpret_cast<const float4*>(ap + 4);
            u32x4 p;
            p[0] = pack2(x0.x, x0.y);
            p[1] = pack2(x0.z, x0.w);
            p[2] = pack2(x1.x, x1.y);
            p[3] = pack2(x1.z, x1.w);
            a = __builtin_bit_cast(bf16x8, p);
        } else {
            const bf16_t* ap = static_cast<const bf16_t*>(A) + (size_t)(m0 + rr) * lda + kq + k0;
            a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(ap));
        }
        const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(bp + k0));
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) red[wv][i][lane] = acc[i];
    __syncthreads();
    for (int q = threadIdx.x; q < 1024; q += 256) {
        const int i = q >> 6, l = q & 63;
        const float s = ((red[0][i][l] + red[1][i][l]) + red[2][i][l]) + red[3][i][l];
        const int row = m0 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
        const int col = n0 + (l & 31);
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

// out[col] = sum_{row < rows} src[row][col] (times [mask > 0] when mask is
// given); 32 columns per workgroup, 8 row groups summed in a fixed order.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ src, const float* __restrict__ mask,
                                                int rows, int ld, float* __restrict__ out) {
    __shared__ float part[8][32];
    const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int col = blockIdx.x * 32 + c;
    float s = 0.0f;
    for (int r = g; r < rows; r += 8) {
        const size_t i = (size_t)r * ld + col;
        const float v = src[i];
        s += (!mask || mask[i] > 0.0f) ? v : 0.0f;
    }
    part[g][c] = s;
    __syncthreads();
    if (g == 0) {
        float t = 0.0f;
        for (int q = 0; q < 8; ++q) t += part[q][c];
        out[col] = t;
    }
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
// Mode profiles <-> network rows.
namespace {

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

struct PackArgs {
    const double* y;  // profiles to precondition: pair p at y + p * pstride (external layout)
    const double* z;  // targets (training) or null
    long pstride;     // doubles between consecutive pairs
    int N, M, nk, K, mp;
    double alpha;
    int p6, din;
    int rows;    // pairs * M * nk
    float* X;    // [rows][din]
    float* T;    // [rows][p6] or null
    float* om;   // [rows] squared RMS s^2, or null
    double* sc;  // [rows][3] (s, Re e, Im e), or null
};

// One wave per row (pair p, mode q = mi * nk + kk).  With y_c(n) the mode's
// profile (c = r, theta, z): s = sqrt(sum |y|^2 / 3N), rho = sum y,
// e = rho / |rho| (1 when |rho| <= 1e-8 3N s), yhat = conj(e) y / s;
// row = [Re, Im of yhat_c(n) at 2(cN + n)], zeros to p6, then the features.
// Target row: conj(e) z / s + yhat.  Rows with s = 0 have zero profile parts.
__global__ __launch_bounds__(256) void k_pack(PackArgs a) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= a.rows) return;
    const int mnk = a.M * a.nk;
    const int p = row / mnk, q = row % mnk;
    const int mi = q / a.nk, kk = q % a.nk;
    const long S = (long)mnk * a.N;
    const double* yb = a.y + (long)p * a.pstride;
    const double* zb = a.z ? a.z + (long)p * a.pstride : nullptr;
    const int n3 = 3 * a.N;
    double s2 = 0.0, rr = 0.0, ri = 0.0;
    for (int e = lane; e < n3; e += 64) {
        const int c = e / a.N, n = e % a.N;
        const long idx = c * S + (long)q * a.N + n;
        const double re = yb[2 * idx], im = yb[2 * idx + 1];
        s2 += re * re + im * im;
        rr += re;
        ri += im;
    }
    s2 = wave_sum(s2);
    rr = wave_sum(rr);
    ri = wave_sum(ri);
    const double s = sqrt(s2 / n3);
    const double rho = sqrt(rr * rr + ri * ri);
    double er = 1.0, ei = 0.0;
    if (rho > 1e-8 * n3 * s) {
        er = rr / rho;
        ei = ri / rho;
    }
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    float* xr = a.X + (long)row * a.din;
    float* tr = a.T ? a.T + (long)row * a.p6 : nullptr;
    for (int e = lane; e < n3; e += 64) {
        const int c = e / a.N, n = e % a.N;
        const long idx = c * S + (long)q * a.N + n;
        const double re = yb[2 * idx], im = yb[2 * idx + 1];
        const double hr = (er * re + ei * im) * inv, hi = (er * im - ei * re) * inv;
        xr[2 * e] = (float)hr;
        xr[2 * e + 1] = (float)hi;
        if (tr) {
            const double zr = zb[2 * idx], zi = zb[2 * idx + 1];
            tr[2 * e] = (float)((er * zr + ei * zi) * inv + hr);
            tr[2 * e + 1] = (float)((er * zi - ei * zr) * inv + hi);
        }
    }
    for (int j = 2 * n3 + lane; j < a.p6; j += 64) {
        xr[j] = 0.0f;
        if (tr) tr[j] = 0.0f;
    }
    for (int j = lane; j < a.din - a.p6; j += 64)
        xr[a.p6 + j] = j < NCOND ? cond_feature(j, mi, kk - (a.K - 1), a.mp, a.alpha) : 0.0f;
    if (lane == 0) {
        if (a.om) a.om[row] = (float)(s * s);
        if (a.sc) {
            a.sc[3 * row] = s;
            a.sc[3 * row + 1] = er;
            a.sc[3 * row + 2] = ei;
        }
    }
}

// z = s e f - y per mode, f the network output read as a complex profile;
// (m = 0, k < 0) is the conjugate of (0, -k).
__global__ void k_unpack(const float* __restrict__ F, int dout, const double* __restrict__ sc,
                         const double* __restrict__ y, double* __restrict__ z, int N, int M, int nk, int K) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    const long S = (long)M * nk * N;
    if (i >= 3 * S) return;
    const int c = (int)(i / S);
    const long rem = i % S;
    const int n = (int)(rem % N);
    const int q0 = (int)(rem / N);
    const int mi = q0 / nk, kk = q0 % nk;
    const bool mir = mi == 0 && kk < K - 1;
    const int q = mir ? 2 * (K - 1) - kk : q0;
    const double s = sc[3 * q], er = sc[3 * q + 1], ei = sc[3 * q + 2];
    const long src = c * S + (long)q * N + n;
    const float* f = F + (long)q * dout + 2 * (c * N + n);
    const double fr = f[0], fi = f[1];
    const double wr = s * (er * fr - ei * fi) - y[2 * src];
    const double wi = s * (er * fi + ei * fr) - y[2 * src + 1];
    z[2 * i] = wr;
    z[2 * i + 1] = mir ? -wi : wi;
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
    int H = 0, L = 0, p6 = 0, din = 0, dout = 0, R = 0;
    long np = 0;
    Segs segs{};
    long woff[MAXL + 2] = {}, boff[MAXL + 2] = {};
    float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    long t = 0;
    float *P = nullptr, *G = nullptr, *Am = nullptr, *Av = nullptr;
    bf16_t *Wb = nullptr, *Wt = nullptr;
    bf16_t *Xb = nullptr, *XT = nullptr;
    float* Hf = nullptr;
    bf16_t *Hb = nullptr, *HT = nullptr;
    float *Z = nullptr, *Y = nullptr, *dH = nullptr;
    bf16_t *dYb = nullptr, *dYT = nullptr, *dZb0 = nullptr, *dZb1 = nullptr, *dZT = nullptr;
    float* X = nullptr;
    double* sc = nullptr;
    float *lrow = nullptr, *wsum = nullptr, *losses = nullptr;
    int loss_cap = 0;
    std::string err;

    float* hf(int l) const { return Hf + (size_t)l * R * H; }
    bf16_t* hb(int l) const { return Hb + (size_t)l * R * H; }
    bf16_t* ht(int l) const { return HT + (size_t)l * H * R; }
    float* z(int l) const { return Z + (size_t)l * R * H; }
};

namespace {

constexpr int LOSS_CAP = 1 << 16;

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
    m->p6 = round32(6 * m->N);
    m->din = m->p6 + NCOND;
    m->dout = m->p6;
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
    lay.take(R * m->din * 4);                      // X
    lay.take(R * 3 * 8);                           // sc
    lay.take(R * 4);                               // lrow
    lay.take(256);                                 // wsum
    lay.take((size_t)LOSS_CAP * 4);                // losses
    return lay;
}

opf_status check_cfg(const opf_ctx* c, const opf_mlp_config* cfg, std::string* why) {
    if (!c || !cfg) return OPF_E_INVALID;
    const opf_params& p = ctx_params(c);
    if (cfg->width < 32 || cfg->width > 512 || cfg->width % 32) {
        if (why) *why = "width must be a multiple of 32 in [32, 512]";
        return OPF_E_INVALID;
    }
    if (cfg->layers < 1 || cfg->layers > MAXL) {
        if (why) *why = "layers must be in [1, 8]";
        return OPF_E_INVALID;
    }
    if (cfg->max_rows < p.M * (2 * p.K - 1) || cfg->max_rows > (1 << 20)) {
        if (why) *why = "max_rows must cover M(2K-1) rows and be <= 2^20";
        return OPF_E_INVALID;
    }
    if (!(cfg->lr >= 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
        !(cfg->adam_eps > 0.0f)) {
        if (why) *why = "bad Adam parameters";
        return OPF_E_INVALID;
    }
    return OPF_OK;
}

template <bool AF32>
hipError_t gemm(hipStream_t s, const void* A, int lda, const bf16_t* B, int ldb, int rows, int cols, int K,
                const Epi& e) {
    if (rows % GT || cols % GT || K % 16 || lda % 8 || ldb % 8 || rows <= 0 || cols <= 0 || K <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm<AF32>, dim3(cols / GT, rows / GT), dim3(256), 0, s, A, lda, B, ldb, K, e);
    return hipGetLastError();
}

// Forward pass over rp rows (multiple of 32) of A (FP32 or bfloat16 rows
// of din).  train: also keep pre-activations and transposed activations.
hipError_t forward(opf_mlp* m, const void* A, bool af32, int lda, int rp, bool train) {
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
    hipError_t st = af32 ? gemm<true>(m->s, A, lda, m->Wb + m->woff[0], m->din, rp, H, m->din, e)
                         : gemm<false>(m->s, A, lda, m->Wb + m->woff[0], m->din, rp, H, m->din, e);
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
        st = gemm<false>(m->s, m->hb(l), H, m->Wb + m->woff[l + 1], H, rp, H, H, f);
        if (st != hipSuccess) return st;
    }
    Epi g{};
    g.bias = m->P + m->boff[L + 1];
    g.out = m->Y;
    g.ldo = m->dout;
    return gemm<false>(m->s, m->hb(L), H, m->Wb + m->woff[L + 1], H, rp, m->dout, H, g);
}

// Loss and parameter gradients after forward(train = true) over rp rows of
// which the first nrows are live; targets t [nrows][dout], weights om.
hipError_t backward(opf_mlp* m, const float* t, const float* om, int nrows, int rp, float* loss_slot) {
    const int H = m->H, L = m->L, R = m->R, dout = m->dout;
    hipStream_t s = m->s;
    hipLaunchKernelGGL(k_weight_sum, dim3(1), dim3(256), 0, s, om, nrows, m->wsum);
    hipLaunchKernelGGL(k_loss, dim3(rp / 4), dim3(256), 0, s, m->Y, t, om, m->wsum, nrows, rp, dout, m->dYb,
                       m->dYT, R, m->lrow);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, m->lrow, nrows, m->wsum, loss_slot);
    hipError_t st = hipGetLastError();
    if (st != hipSuccess) return st;
    {  // output layer: dW = dY^T H_L, db = colsum dY, dH_L = dY W_out
        Epi e{};
        e.out = m->G + m->woff[L + 1];
        e.ldo = H;
        if ((st = gemm<false>(s, m->dYT, R, m->ht(L), R, dout, H, rp, e)) != hipSuccess) return st;
        hipLaunchKernelGGL(k_colsum, dim3(dout / 32), dim3(256), 0, s, m->Y, nullptr, rp, dout,
                           m->G + m->boff[L + 1]);
        Epi f{};
        f.out = m->dH;
        f.ldo = H;
        f.mask = m->z(L - 1);
        f.ldm = H;
        f.outb = m->dZb0;
        f.ldb = H;
        f.outT = m->dZT;
        f.ldt = R;
        if ((st = gemm<false>(s, m->dYb, dout, m->Wt + m->woff[L + 1], dout, rp, H, dout, f)) != hipSuccess)
            return st;
    }
    bf16_t* dz[2] = {m->dZb0, m->dZb1};
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        // dz_l = dH_{l+1} [z_l > 0] is in dz[cur] (row-major) and dZT (transposed)
        hipLaunchKernelGGL(k_colsum, dim3(H / 32), dim3(256), 0, s, m->dH, m->z(l), rp, H, m->G + m->boff[l + 1]);
        Epi e{};
        e.out = m->G + m->woff[l + 1];
        e.ldo = H;
        if ((st = gemm<false>(s, m->dZT, R, m->ht(l), R, H, H, rp, e)) != hipSuccess) return st;
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
        if ((st = gemm<false>(s, dz[cur], H, m->Wt + m->woff[l + 1], H, rp, H, H, f)) != hipSuccess) return st;
        cur ^= 1;
    }
    // input layer: dW_in = dH_0^T X, db_in = colsum dH_0
    hipLaunchKernelGGL(k_colsum, dim3(H / 32), dim3(256), 0, s, m->dH, nullptr, rp, H, m->G + m->boff[0]);
    Epi e{};
    e.out = m->G + m->woff[0];
    e.ldo = m->din;
    if ((st = gemm<false>(s, m->dZT, R, m->XT, R, H, m->din, rp, e)) != hipSuccess) return st;
    return hipGetLastError();
}

hipError_t adam(opf_mlp* m) {
    m->t += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)m->b1, (double)m->t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)m->b2, (double)m->t)));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((m->np + 255) / 256)), dim3(256), 0, m->s, m->P, m->G, m->Am, m->Av,
                       m->np, m->lr, m->b1, m->b2, c1, c2, m->eps, m->segs, m->Wb, m->Wt);
    return hipGetLastError();
}

hipError_t rows_bf16(opf_mlp* m, const float* x, int nrows, int rp, bool transposed) {
    const size_t n = (size_t)rp * m->din;
    hipLaunchKernelGGL(k_rows_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->s, x, nrows, rp, m->din,
                       m->Xb, transposed ? m->XT : nullptr, m->R);
    return hipGetLastError();
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
    cfg->max_rows = 0;
    cfg->seed = 1;
    cfg->lr = 1e-3f;
    cfg->beta1 = 0.9f;
    cfg->beta2 = 0.999f;
    cfg->adam_eps = 1e-8f;
    return OPF_OK;
}

opf_status opf_mlp_workspace_size(const opf_ctx* ctx, const opf_mlp_config* cfg, size_t* bytes) {
    if (!bytes) return OPF_E_INVALID;
    const opf_status st = check_cfg(ctx, cfg, nullptr);
    if (st != OPF_OK) return st;
    opf_mlp m;
    const opf_params& p = ctx_params(ctx);
    m.N = p.N;
    m.H = cfg->width;
    m.L = cfg->layers;
    m.R = round32(cfg->max_rows);
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
    const opf_params& p = ctx_params(ctx);
    m->ctx = ctx;
    m->s = ctx_stream(ctx);
    m->N = p.N;
    m->M = p.M;
    m->K = p.K;
    m->nk = 2 * p.K - 1;
    m->mp = p.mp;
    m->alpha = p.alpha;
    m->H = cfg->width;
    m->L = cfg->layers;
    m->R = round32(cfg->max_rows);
    m->lr = cfg->lr;
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
    at(m->X);
    at(m->sc);
    at(m->lrow);
    at(m->wsum);
    at(m->losses);
    m->loss_cap = LOSS_CAP;
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
    // rows past M(2K-1) of the preconditioner input stay zero
    if (hipMemsetAsync(m->X, 0, (size_t)m->R * m->din * 4, m->s) != hipSuccess ||
        hipStreamSynchronize(m->s) != hipSuccess) {
        delete m;
        return OPF_E_HIP;
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
    MCHK(net, forward(net, net->Xb, false, net->din, rp, false));
    MCHK(net, hipMemcpyAsync(y_dev, net->Y, (size_t)rows * net->dout * 4, hipMemcpyDeviceToDevice, net->s));
    return OPF_OK;
}

opf_status opf_mlp_gradient(opf_mlp* net, const float* x_dev, const float* t_dev, const float* w_dev, int32_t rows,
                            double* loss_host, float* grad_host) {
    if (!net || !x_dev || !t_dev || rows < 1 || rows > net->R) return OPF_E_INVALID;
    const int rp = round32(rows);
    MCHK(net, rows_bf16(net, x_dev, rows, rp, true));
    MCHK(net, forward(net, net->Xb, false, net->din, rp, true));
    MCHK(net, backward(net, t_dev, w_dev, rows, rp, net->losses));
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
            MCHK(net, forward(net, net->Xb, false, net->din, rp, true));
            MCHK(net, backward(net, t_dev + (size_t)r0 * net->dout, w_dev ? w_dev + r0 : nullptr, n, rp,
                               net->losses + step));
            MCHK(net, adam(net));
            ++step;
        }
    }
    if (loss_host && epochs > 0) {
        std::vector<float> l(step);
        MCHK(net, hipMemcpyAsync(l.data(), net->losses, (size_t)step * 4, hipMemcpyDeviceToHost, net->s));
        MCHK(net, hipStreamSynchronize(net->s));
        for (int ep = 0; ep < epochs; ++ep) {
            double a = 0.0;
            for (int i = 0; i < nb; ++i) a += l[(size_t)ep * nb + i];
            loss_host[ep] = (float)(a / nb);
        }
    } else {
        MCHK(net, hipStreamSynchronize(net->s));
    }
    return OPF_OK;
}

opf_status opf_mlp_pack_pairs(opf_ctx* ctx, const opf_mlp* net, const void* pairs_dev, int32_t npairs, float* x_dev,
                              float* t_dev, float* w_dev) {
    if (!ctx || !net || !pairs_dev || npairs < 1 || !x_dev || !t_dev) return OPF_E_INVALID;
    if (!same_grid(net, ctx)) return OPF_E_INVALID;
    const long vec = 2L * 3 * net->M * net->nk * net->N;  // doubles per vector
    PackArgs a{};
    a.z = static_cast<const double*>(pairs_dev);
    a.y = a.z + vec;
    a.pstride = 2 * vec;
    a.N = net->N;
    a.M = net->M;
    a.nk = net->nk;
    a.K = net->K;
    a.mp = net->mp;
    a.alpha = net->alpha;
    a.p6 = net->p6;
    a.din = net->din;
    a.rows = npairs * net->M * net->nk;
    a.X = x_dev;
    a.T = t_dev;
    a.om = w_dev;
    hipLaunchKernelGGL(k_pack, dim3((a.rows + 3) / 4), dim3(256), 0, ctx_stream(ctx), a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        ctx_set_error(ctx, std::string("k_pack: ") + hipGetErrorString(e));
        return OPF_E_HIP;
    }
    return OPF_OK;
}

opf_status opf_precondition(opf_ctx* ctx, opf_mlp* net, const void* v_dev, void* z_dev) {
    if (!ctx || !net || !v_dev || !z_dev) return OPF_E_INVALID;
    if (!same_grid(net, ctx)) return OPF_E_INVALID;
    const int rows = net->M * net->nk;
    PackArgs a{};
    a.y = static_cast<const double*>(v_dev);
    a.N = net->N;
    a.M = net->M;
    a.nk = net->nk;
    a.K = net->K;
    a.mp = net->mp;
    a.alpha = net->alpha;
    a.p6 = net->p6;
    a.din = net->din;
    a.rows = rows;
    a.X = net->X;
    a.sc = net->sc;
    hipLaunchKernelGGL(k_pack, dim3((rows + 3) / 4), dim3(256), 0, net->s, a);
    MCHK(net, hipGetLastError());
    MCHK(net, forward(net, net->X, true, net->din, round32(rows), false));
    const long n = 3L * rows * net->N;
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, net->s, net->Y, net->dout, net->sc,
                       static_cast<const double*>(v_dev), static_cast<double*>(z_dev), net->N, net->M, net->nk,
                       net->K);
    MCHK(net, hipGetLastError());
    return OPF_OK;
}

const char* opf_mlp_last_error(const opf_mlp* net) { return net ? net->err.c_str() : "null network"; }

}  // extern "C"
