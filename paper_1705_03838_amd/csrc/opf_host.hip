// Host side of the pipe-flow time-step library: C ABI, create-time tables
// (nodes, finite-difference weights, quadrature, banded LU factors,
// influence-matrix data, FFT twiddles), workspace layout and the captured
// step graph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "opf_internal.h"

using namespace opf;
using cd = std::complex<double>;

struct opf_ctx {
    opf_params p{};
    std::vector<double> r, rinv, quad, d1, d2;  // host copies
    std::vector<int> s0;
    int nk = 0, MU = 0, nfac = 0, gm = 1;
    int tz = DEFAULT_TZ, ztile = DEFAULT_ZTILE;  // transform tile shapes
    int narrow = 0;  // see SolveArgs::narrow
    double qG_inv = 0.0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    hipGraphExec_t graph = nullptr;   // one step
    hipGraphExec_t graphs = nullptr;  // STEP_GRAPH_STEPS steps
    unsigned char* ws = nullptr;
    size_t ws_bytes = 0;
    Tables t{};
    // buffers (device)
    double *u = nullptr, *up = nullptr, *w64 = nullptr, *beta = nullptr, *partial = nullptr;
    double *dpart = nullptr, *cflw = nullptr, *cpart = nullptr;  // diagnostics: per-mode g / div, CFL weights, per-block CFL
    void *w = nullptr, *Nn = nullptr, *Np = nullptr, *H = nullptr, *G = nullptr;
    float *u32 = nullptr, *up32 = nullptr;
    void *twz = nullptr, *twt = nullptr;
    bool have_state = false;
    bool pc_valid = false;  // up / up32 hold the iterate before the last corrector of the last step
    bool in_ensemble = false;  // member of an ensemble: its step runs in the class graph, dt is fixed
    double rot[3] = {0.0, 0.0, 0.0};  // Coriolis rotation vector (opf_set_rotation)
    double* wall = nullptr;           // wall velocity [3][M][nk] complex in the workspace
    bool has_wall = false;            // opf_set_wall_velocity set a moving wall
    std::string err;
};

namespace opf {
hipStream_t ctx_stream(const opf_ctx* c) { return c->stream; }
const opf_params& ctx_params(const opf_ctx* c) { return c->p; }
void ctx_set_error(opf_ctx* c, const std::string& msg) { c->err = msg; }
}  // namespace opf

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// ---- parameter checks ---------------------------------------------------
bool factor23(int L) {
    if (L <= 0) return false;
    while (L % 2 == 0) L /= 2;
    while (L % 3 == 0) L /= 3;
    return L == 1;
}

opf_status validate(const opf_params* p, std::string* why) {
    auto bad = [&](const char* s) { if (why) *why = s; return OPF_E_INVALID; };
    if (!p) return bad("null parameters");
    if (p->stencil != W9) return bad("stencil must be 9");
    if (p->N < 12) return bad("N must be >= 12");
    if (p->N > NMAX) { if (why) *why = "N > 64 not supported"; return OPF_E_UNSUPPORTED; }
    if (p->M < 2 || p->K < 2 || p->M > 64 || p->K > 64) return bad("M and K must be in [2, 64]");
    if (!factor23(3 * p->M) || !factor23(3 * p->K) || !nonlinear_supported(p->M, p->K)) {
        if (why) *why = "3M and 3K must be supported FFT lengths (2^a 3^b <= 192)";
        return OPF_E_UNSUPPORTED;
    }
    if (p->mp < 1) return bad("mp must be >= 1");
    if (!(p->alpha > 0) || !(p->Re > 0) || !(p->dt > 0)) return bad("alpha, Re, dt must be > 0");
    if (!(p->c > 0 && p->c <= 1)) return bad("c must be in (0, 1]");
    if (p->n_corr < 1) return bad("n_corr must be >= 1");
    if (p->precision != OPF_FP64 && p->precision != OPF_MIXED) return bad("unknown precision");
    if (p->r_nodes) {
        const double* r = p->r_nodes;
        if (!(r[0] > 0) || r[p->N - 1] != 1.0) return bad("nodes must lie in (0,1] with r[N-1] = 1");
        for (int i = 1; i < p->N; ++i)
            if (!(r[i] > r[i - 1])) return bad("nodes must increase");
    }
    return OPF_OK;
}

// ---- finite-difference weights (Fornberg's recursion, Math. Comp. 51, 1988)
// Weights c[d][j] with f^(d)(z) ~ sum_j c[d][j] f(x_j), d <= 2.
void fornberg(double z, const double* x, int n, double c[3][W9]) {
    for (int d = 0; d < 3; ++d)
        for (int j = 0; j < n; ++j) c[d][j] = 0.0;
    double c1 = 1.0, c4 = x[0] - z;
    c[0][0] = 1.0;
    for (int i = 1; i < n; ++i) {
        const int mn = std::min(i, 2);
        double c2 = 1.0;
        const double c5 = c4;
        c4 = x[i] - z;
        for (int j = 0; j < i; ++j) {
            const double c3 = x[i] - x[j];
            c2 *= c3;
            if (j == i - 1) {
                for (int d = mn; d >= 1; --d) c[d][i] = c1 * (d * c[d - 1][i - 1] - c5 * c[d][i - 1]) / c2;
                c[0][i] = -c1 * c5 * c[0][i - 1] / c2;
            }
            for (int d = mn; d >= 1; --d) c[d][j] = (c4 * c[d][j] - d * c[d - 1][j]) / c3;
            c[0][j] = c4 * c[0][j] / c3;
        }
        c1 = c2;
    }
}

// Extended node: index e >= 0 is r[e]; e < 0 is the mirror point -r[-e-1].
double ext(const std::vector<double>& r, int e) { return e >= 0 ? r[e] : -r[-e - 1]; }
int window_start(int n, int N) { return std::min(n - HALF, N - W9); }

// Gauss-Legendre nodes / weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}


// Nodes, folded finite-difference weights and quadrature (host, create time).
void build_grid(opf_ctx* c, const double* r_nodes) {
    const int N = c->p.N;
    // nodes (default: positive Gauss-Lobatto points of T_{2N-1})
    c->r.resize(N);
    for (int n = 0; n < N; ++n)
        c->r[n] = r_nodes ? r_nodes[n] : std::cos(M_PI * (N - 1 - n) / (2.0 * N - 1.0));
    c->rinv.resize(N);
    for (int n = 0; n < N; ++n) c->rinv[n] = 1.0 / c->r[n];

    // finite-difference weights folded onto nodes with axis parity
    c->s0.resize(N);
    c->d1.assign(2 * N * W9, 0.0);
    c->d2.assign(2 * N * W9, 0.0);
    for (int n = 0; n < N; ++n) {
        const int e0 = window_start(n, N);
        c->s0[n] = std::max(e0, 0);
        double x[W9], w[3][W9];
        for (int j = 0; j < W9; ++j) x[j] = ext(c->r, e0 + j);
        fornberg(c->r[n], x, W9, w);
        for (int par = 0; par < 2; ++par) {
            const double sgn = par == 0 ? 1.0 : -1.0;
            for (int j = 0; j < W9; ++j) {
                const int e = e0 + j;
                const int col = e >= 0 ? e : -e - 1;
                const double f = e >= 0 ? 1.0 : sgn;
                c->d1[(par * N + n) * W9 + (col - c->s0[n])] += f * w[1][j];
                c->d2[(par * N + n) * W9 + (col - c->s0[n])] += f * w[2][j];
            }
        }
    }
    // Row i of every radial operator is zero left of column s0[i] (the wall
    // row is the identity), and LU without pivoting fills nothing left of a
    // row's first nonzero.  So L[i][j] != 0 with i > j + 4 needs a row with
    // s0[i] <= j <= i - 5, and columns before the smallest such s0[i] have at
    // most four nonzero entries below the diagonal.
    c->narrow = N;
    for (int i = 0; i < N - 1; ++i)
        if (c->s0[i] <= i - 5) c->narrow = std::min(c->narrow, c->s0[i]);

    // quadrature: exact integral of each interval's stencil interpolant times r
    {
        std::vector<double> gx, gw;
        gauss_legendre(8, gx, gw);
        c->quad.assign(N, 0.0);
        for (int j = 0; j < N; ++j) {
            const double lo = j == 0 ? 0.0 : c->r[j - 1], hi = c->r[j];
            const int e0 = window_start(j, N);
            double x[W9], w[3][W9];
            for (int i = 0; i < W9; ++i) x[i] = ext(c->r, e0 + i);
            for (int q = 0; q < 8; ++q) {
                const double rq = 0.5 * (hi - lo) * gx[q] + 0.5 * (hi + lo);
                const double wq = 0.5 * (hi - lo) * gw[q] * rq;
                fornberg(rq, x, W9, w);  // w[0] = Lagrange basis values at rq
                for (int i = 0; i < W9; ++i) {
                    const int e = e0 + i;
                    c->quad[e >= 0 ? e : -e - 1] += wq * w[0][i];
                }
            }
        }
    }

}

struct Layout {
    size_t r, rinv, quad, d1, d2, wl, s0, fac, img, dinv, hom, ainv, green, flags, qg, wall, twz, twt;
    size_t u, up, w64, w, Nn, Np, H, G, u32, up32, beta, partial, dpart, cflw, cpart, total;
};

Layout layout(const opf_params& p) {
    const size_t N = p.N, M = p.M, K = p.K, nk = 2 * K - 1;
    const size_t MU = (size_t)p.mp * (M - 1) + 2;
    const size_t nfac = MU * K + M * K;
    const size_t S = M * nk * N;  // complex entries per field
    const size_t Hn = N * M * 3 * K;
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    L.r = take(N * 8);
    L.rinv = take(N * 8);
    L.quad = take(N * 8);
    L.d1 = take(2 * N * W9 * 8);
    L.d2 = take(2 * N * W9 * 8);
    L.wl = take(2 * N * W9 * 8);
    L.s0 = take(N * 4);
    L.fac = take(nfac * N * FACW * 8);
    // substitution images at the largest size (no narrow rows)
    L.img = take(nfac * solve_image_doubles(solve_nb((int)N), 0) * 8);
    L.dinv = take(nfac * solve_nb((int)N) * 8);
    L.hom = take(M * K * NHOM * N * 8);
    L.ainv = take(M * nk * 16 * 16);
    L.green = take(N * 8);
    L.flags = take((nfac + M * nk) * 4);
    L.qg = take(8);
    L.wall = take(3 * M * nk * 16);
    L.twz = take(3 * K * 16);
    L.twt = take(3 * M * 16);
    L.u = take(3 * S * 16);
    L.up = take(3 * S * 16);
    L.w64 = take(3 * S * 16);
    L.w = take(3 * S * 16);
    L.Nn = take(3 * S * 16);
    L.Np = take(3 * S * 16);
    L.H = take(6 * Hn * 16);
    L.G = take(3 * Hn * 16);
    L.u32 = take(3 * S * 8);
    L.up32 = take(3 * S * 8);
    L.beta = take(8);
    L.partial = take(2 * M * 8);
    L.dpart = take(2 * M * nk * 8);
    L.cflw = take(2 * N * 8);
    L.cpart = take(N * ((3 * K + 3) / 4) * 8);
    L.total = o;
    return L;
}

#define HIPCHK(ctx, call)                                                               \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);             \
            return OPF_E_HIP;                                                           \
        }                                                                               \
    } while (0)

template <typename T>
__global__ void k_convert(const double* __restrict__ in, T* __restrict__ out, size_t n) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = T(in[i]);
}
__global__ void k_widen(const float* __restrict__ in, double* __restrict__ out, size_t n) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = double(in[i]);
}

// F = shift(u, -s) - x: F_k = u_k exp(+i alpha k s) - x_k (complex128 external layout).
__global__ void k_shift_sub(const double* __restrict__ u, const double* __restrict__ x, double* __restrict__ F,
                            int N, int nk, int K, size_t total, double alpha, double sft) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int kk = (int)((i / N) % nk);
    const double ph = alpha * (kk - (K - 1)) * sft;
    const double c = cos(ph), sn = sin(ph);
    const double ur = u[2 * i], ui = u[2 * i + 1];
    F[2 * i] = ur * c - ui * sn - x[2 * i];
    F[2 * i + 1] = ur * sn + ui * c - x[2 * i + 1];
}

// Laminar flow u_z(0,0) = 1 - r^2, every other coefficient zero (complex128
// external layout), in u and its FP32 shadow.
__global__ void k_laminar(double* __restrict__ u, float* __restrict__ u32, const double* __restrict__ r, int N,
                          int nk, int K, size_t total) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const size_t S = total / 3, e = i % S;
    const bool lam = i / S == 2 && e / N == (size_t)(K - 1);  // m = 0, k = 0 of u_z
    const double v = lam ? 1.0 - r[e % N] * r[e % N] : 0.0;
    u[2 * i] = v;
    u[2 * i + 1] = 0.0;
    u32[2 * i] = float(v);
    u32[2 * i + 1] = 0.0f;
}

// Axial derivative d_z x: out_k = i alpha k x_k (complex128 external layout).
__global__ void k_ddz(const double* __restrict__ x, double* __restrict__ out, int N, int nk, int K, size_t total,
                      double alpha) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const double ka = alpha * ((int)((i / N) % nk) - (K - 1));
    const double xr = x[2 * i], xi = x[2 * i + 1];
    out[2 * i] = -ka * xi;
    out[2 * i + 1] = ka * xr;
}

// Per-m partial sums of w_n Re(a conj(b)) over components, k and n (the
// energy inner product before the m weights); fixed summation order.
__global__ __launch_bounds__(256) void k_wdot(const double* __restrict__ a, const double* __restrict__ b,
                                              const double* __restrict__ quad, double* __restrict__ partial,
                                              int N, int M, int nk) {
    __shared__ double red[256];
    const int mi = blockIdx.x;
    const size_t S = (size_t)M * nk * N;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nk * N; i += 256) {
        const int n = i % N;
        const size_t off = (size_t)mi * nk * N + i;
        double sum = 0.0;
        for (int c = 0; c < 3; ++c) {
            const size_t j = 2 * (c * S + off);
            sum += a[j] * b[j] + a[j + 1] * b[j + 1];
        }
        acc += quad[n] * sum;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[mi] = red[0];
}

// Per-m partial sums of w_n |a - b|^2 over components, k and n (the squared
// energy norm of a - b before the m weights); b in the working precision.
template <typename T>
__global__ __launch_bounds__(256) void k_pcdiff(const double* __restrict__ a, const T* __restrict__ b,
                                                const double* __restrict__ quad, double* __restrict__ partial,
                                                int N, int M, int nk) {
    __shared__ double red[256];
    const int mi = blockIdx.x;
    const size_t S = (size_t)M * nk * N;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nk * N; i += 256) {
        const int n = i % N;
        const size_t off = (size_t)mi * nk * N + i;
        double sum = 0.0;
        for (int c = 0; c < 3; ++c) {
            const size_t j = 2 * (c * S + off);
            const double dr = a[j] - (double)b[j], di = a[j + 1] - (double)b[j + 1];
            sum += dr * dr + di * di;
        }
        acc += quad[n] * sum;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[mi] = red[0];
}

// y = a x + b y over n doubles.
// y = a x + b y; with b = 0, y is overwritten without being read (a fresh
// buffer may hold NaN, and 0 * NaN is NaN).
__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y, size_t n) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

// Independent unit normals in every real and imaginary part of a field:
// entry i takes two uniforms from SplitMix64 (Steele, Lea & Flood 2014) at
// counters 2i, 2i+1 of the seed's stream and turns them into a pair of
// normals by the Box-Muller transform.
__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__global__ void k_noise(double* __restrict__ z, size_t n, uint64_t seed) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t base = seed + 0x9E3779B97F4A7C15ull * (2 * (uint64_t)i + 1);
    const double u1 = ((double)(mix64(base) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = (double)(mix64(base + 0x9E3779B97F4A7C15ull) >> 11) * (1.0 / 9007199254740992.0);
    const double rad = sqrt(-2.0 * log(u1)), th = 2.0 * M_PI * u2;
    z[2 * i] = rad * cos(th);
    z[2 * i + 1] = rad * sin(th);
}

// Spectrum of a real field at m = 0: A(0, -k) = conj A(0, k), A(0, 0) real.
__global__ void k_realfield(double* __restrict__ z, int N, int M, int nk, int K) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * K * N) return;
    const int c = i / (K * N), kp = (i / N) % K, n = i % N;  // kp = k >= 0
    const size_t S = (size_t)M * nk * N;
    const size_t pos = c * S + (size_t)(K - 1 + kp) * N + n;
    if (kp == 0) {
        z[2 * pos + 1] = 0.0;
        return;
    }
    const size_t neg = c * S + (size_t)(K - 1 - kp) * N + n;
    z[2 * neg] = z[2 * pos];
    z[2 * neg + 1] = -z[2 * pos + 1];
}

hipError_t to_f32(const double* in, float* out, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_convert<float>, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t to_f64(const float* in, double* out, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_widen, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

size_t field_entries(const opf_ctx* c) { return (size_t)c->p.M * c->nk * c->p.N; }

NLArgs nl_args(const opf_ctx* c, const void* u, const void* w, void* out) {
    NLArgs a{};
    a.N = c->p.N;
    a.M = c->p.M;
    a.K = c->p.K;
    a.nk = c->nk;
    const size_t S = field_entries(c);
    const size_t esz = c->p.precision == OPF_MIXED ? 8 : 16;
    for (int f = 0; f < 3; ++f) {
        a.in[f] = static_cast<const unsigned char*>(u) + f * S * esz;
        a.in[3 + f] = static_cast<const unsigned char*>(w) + f * S * esz;
        a.out[f] = static_cast<unsigned char*>(out) + f * S * esz;
    }
    a.H = c->H;
    a.G = c->G;
    a.twz = c->twz;
    a.twt = c->twt;
    a.scale = 1.0 / (9.0 * c->p.K * c->p.M);
    for (int i = 0; i < 3; ++i) a.rot[i] = c->rot[i];
    a.rotating = c->rot[0] != 0.0 || c->rot[1] != 0.0 || c->rot[2] != 0.0;
    a.tz = c->tz;
    a.ztile = c->ztile;
    return a;
}

SolveArgs solve_args(const opf_ctx* c, int kind) {
    SolveArgs a{};
    a.N = c->p.N;
    a.M = c->p.M;
    a.K = c->p.K;
    a.nk = c->nk;
    a.mp = c->p.mp;
    a.MU = c->MU;
    a.gm = c->gm;
    a.narrow = c->narrow;
    a.kind = kind;
    a.fixed_flux = c->p.fixed_flux;
    a.alpha = c->p.alpha;
    a.Re = c->p.Re;
    a.c = c->p.c;
    a.inv_dt = 1.0 / c->p.dt;
    a.aexp = (1.0 - c->p.c) / c->p.Re;
    a.force = 4.0 / c->p.Re;
    a.beta_out = c->beta;
    a.wall = c->has_wall ? c->wall : nullptr;
    a.t = c->t;
    return a;
}

// Operator tables for the current dt, built on the device (with pressure,
// also the dt-independent pressure factors and unit-wall pressures), then
// the status flags and the Green's function integral read back
// (synchronises).  On failure c->err names the table.
opf_status device_tables(opf_ctx* c, bool pressure) {
    const opf_params& p = c->p;
    const Layout Lo = layout(p);
    FactorArgs a{};
    a.N = p.N;
    a.M = p.M;
    a.K = p.K;
    a.MU = c->MU;
    a.mp = p.mp;
    a.alpha = p.alpha;
    a.cr = p.c / p.Re;
    a.inv_dt = 1.0 / p.dt;
    a.rinv = c->t.rinv;
    a.quad = c->t.quad;
    a.d1 = c->t.d1;
    a.d2 = c->t.d2;
    a.s0 = c->t.s0;
    a.fac = reinterpret_cast<double*>(c->ws + Lo.fac);
    a.img = reinterpret_cast<double*>(c->ws + Lo.img);
    a.dinv = reinterpret_cast<double*>(c->ws + Lo.dinv);
    a.NB = solve_nb(p.N);
    a.NW = solve_nw(p.N, c->narrow);
    a.hom = reinterpret_cast<double*>(c->ws + Lo.hom);
    a.ainv = reinterpret_cast<double*>(c->ws + Lo.ainv);
    a.green = reinterpret_cast<double*>(c->ws + Lo.green);
    a.flags = reinterpret_cast<int*>(c->ws + Lo.flags);
    a.qg = reinterpret_cast<double*>(c->ws + Lo.qg);
    HIPCHK(c, launch_operator_tables(a, pressure, c->stream));
    const int nh = c->MU * p.K, np = p.M * p.K, modes = p.M * c->nk;
    std::vector<int> fl(nh + np + modes);
    double qg = 0.0;
    HIPCHK(c, hipMemcpyAsync(fl.data(), a.flags, fl.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&qg, a.qg, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int q = 0; q < nh + np + modes; ++q)
        if (fl[q] != 0 && (q < nh || pressure)) {
            c->err = q < nh ? "Helmholtz factor unstable without pivoting"
                   : q < nh + np ? "pressure factor unstable without pivoting" : "singular influence matrix";
            return OPF_E_NUMERIC;
        }
    if (!(std::isfinite(qg) && qg != 0.0)) {
        c->err = "flux Green's function has no flux";
        return OPF_E_NUMERIC;
    }
    c->qG_inv = 1.0 / qg;
    c->t.qG_inv = c->qG_inv;
    return OPF_OK;
}

// Enqueue one predictor-corrector step (captured into the step graph).
opf_status enqueue_step(opf_ctx* c, hipStream_t s) {
    const bool mixed = c->p.precision == OPF_MIXED;
    const void* uin = mixed ? (const void*)c->u32 : (const void*)c->u;
    const void* upin = mixed ? (const void*)c->up32 : (const void*)c->up;
    if (c->p.nonlinear) HIPCHK(c, launch_nonlinear(nl_args(c, uin, c->w, c->Nn), c->p.precision, s));
    SolveArgs a = solve_args(c, OPF_SOLVE_PRED);
    a.u0 = c->u;
    a.n0 = c->Nn;
    a.u_out = mixed ? nullptr : c->up;
    a.u_out32 = mixed ? c->up32 : nullptr;
    a.w_out = c->w;
    HIPCHK(c, launch_solve(a, c->p.precision, s));
    for (int it = 0; it < c->p.n_corr; ++it) {
        if (c->p.nonlinear) HIPCHK(c, launch_nonlinear(nl_args(c, upin, c->w, c->Np), c->p.precision, s));
        SolveArgs b = solve_args(c, OPF_SOLVE_CORR);
        b.u0 = c->u;
        b.n0 = c->Nn;
        b.n1 = c->Np;
        const bool last = it == c->p.n_corr - 1;
        b.u_out = last ? c->u : (mixed ? nullptr : c->up);
        b.u_out32 = mixed ? (last ? c->u32 : c->up32) : nullptr;
        b.w_out = c->w;
        HIPCHK(c, launch_solve(b, c->p.precision, s));
    }
    return OPF_OK;
}

// omega of the state, and the FP32 shadows in mixed precision.
opf_status refresh_derived(opf_ctx* c) {
    const size_t n = 2 * 3 * field_entries(c);
    AuxArgs x{};
    x.N = c->p.N;
    x.M = c->p.M;
    x.K = c->p.K;
    x.nk = c->nk;
    x.mp = c->p.mp;
    x.alpha = c->p.alpha;
    x.u = c->u;
    x.t = c->t;
    x.mirror = 1;
    if (c->p.precision == OPF_MIXED) {
        x.w = c->w64;
        HIPCHK(c, launch_vorticity(x, c->stream));
        HIPCHK(c, to_f32(c->w64, static_cast<float*>(c->w), n, c->stream));
        HIPCHK(c, to_f32(c->u, c->u32, n, c->stream));
    } else {
        x.w = static_cast<double*>(c->w);
        HIPCHK(c, launch_vorticity(x, c->stream));
    }
    return OPF_OK;
}

// CFL: z-inverse transform of the state's velocity and vorticity (the H
// buffer), then per-block maxima over the theta-inverse velocity lines of
// |u_r|/dr + |u_theta|/(r dtheta) + |u_z|/dz into cpart.
hipError_t enqueue_cfl(opf_ctx* c) {
    const int N = c->p.N, K = c->p.K;
    const bool mixed = c->p.precision == OPF_MIXED;
    const NLArgs nl = nl_args(c, mixed ? (const void*)c->u32 : (const void*)c->u, c->w, c->Nn);
    hipError_t he = launch_nonlinear_stage(nl, c->p.precision, 0, c->stream);
    if (he != hipSuccess) return he;
    return launch_cfl(nl, c->p.precision, c->cflw, c->cflw + N, c->p.alpha * 3 * K / (2.0 * M_PI), c->cpart,
                      c->stream);
}
size_t cfl_parts(const opf_ctx* c) { return (size_t)c->p.N * ((3 * c->p.K + 3) / 4); }

// Per-m partial sums of the last correction into partial[0..M).
hipError_t enqueue_pcdiff(opf_ctx* c) {
    const int M = c->p.M;
    if (c->p.precision == OPF_MIXED)
        hipLaunchKernelGGL(k_pcdiff<float>, dim3(M), dim3(256), 0, c->stream, c->u, c->up32, c->t.quad,
                           c->partial, c->p.N, M, c->nk);
    else
        hipLaunchKernelGGL(k_pcdiff<double>, dim3(M), dim3(256), 0, c->stream, c->u, c->up, c->t.quad,
                           c->partial, c->p.N, M, c->nk);
    return hipGetLastError();
}
double weighted_norm(const std::vector<double>& part) {
    double s = 0.0;
    for (size_t m = 0; m < part.size(); ++m) s += (m == 0 ? 1.0 : 2.0) * part[m];
    return std::sqrt(s);
}

// The step size after a check (the rule declared with opf_dt_control); a
// value below dt_min is returned as is and rejected by the caller.
double next_dt(double dt, double cfl, double delta, const opf_dt_control& k) {
    const double U = cfl / dt;
    const double dt_c = U > 0 ? k.courant / U : INFINITY;
    const double dt_e = k.pc_tol > 0 && delta > 0 ? dt * std::sqrt(k.pc_tol / delta) : INFINITY;
    const double lim = std::min(dt_c, dt_e);
    const double nw = std::min(k.dt_max, lim / (1.0 + k.grow));
    if (nw < k.dt_min) return nw;
    if (dt > lim) return nw;
    if (nw > dt && (nw >= (1.0 + k.grow) * dt || nw == k.dt_max)) return nw;
    return dt;
}

}  // namespace

extern "C" {

const char* opf_status_string(opf_status s) {
    switch (s) {
        case OPF_OK: return "ok";
        case OPF_E_INVALID: return "invalid argument";
        case OPF_E_NOMEM: return "workspace too small";
        case OPF_E_HIP: return "HIP runtime error";
        case OPF_E_UNSUPPORTED: return "unsupported size or option";
        case OPF_E_NUMERIC: return "numerical failure";
        case OPF_E_STATE: return "no state set";
    }
    return "unknown status";
}

const char* opf_last_error(const opf_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

opf_status opf_default_params(opf_params* p) {
    if (!p) return OPF_E_INVALID;
    *p = opf_params{};
    p->N = 24;
    p->M = 8;
    p->K = 8;
    p->mp = 1;
    p->stencil = 9;
    p->alpha = 1.25;
    p->Re = 2400.0;
    p->dt = 0.01;
    p->c = 0.5;
    p->n_corr = 1;
    p->fixed_flux = 1;
    p->precision = OPF_FP64;
    p->nonlinear = 1;
    p->r_nodes = nullptr;
    return OPF_OK;
}

opf_status opf_tables(const opf_params* p, double* r, double* quad, double* d1, double* d2, int32_t* s0) {
    const opf_status st = validate(p, nullptr);
    if (st != OPF_OK) return st;
    opf_ctx c;
    c.p = *p;
    build_grid(&c, p->r_nodes);
    const int N = p->N;
    if (r) std::copy(c.r.begin(), c.r.end(), r);
    if (quad) std::copy(c.quad.begin(), c.quad.end(), quad);
    if (d1) std::copy(c.d1.begin(), c.d1.end(), d1);
    if (d2) std::copy(c.d2.begin(), c.d2.end(), d2);
    if (s0) for (int n = 0; n < N; ++n) s0[n] = c.s0[n];
    return OPF_OK;
}

opf_status opf_workspace_size(const opf_params* p, size_t* bytes) {
    if (!bytes) return OPF_E_INVALID;
    const opf_status st = validate(p, nullptr);
    if (st != OPF_OK) return st;
    *bytes = layout(*p).total;
    return OPF_OK;
}

opf_status opf_create(const opf_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                      opf_ctx** out) {
    if (!out) return OPF_E_INVALID;
    *out = nullptr;
    std::string why;
    const opf_status st = validate(p, &why);
    if (st != OPF_OK) return st;
    const Layout Lo = layout(*p);
    if (!dev_workspace || bytes < Lo.total) return OPF_E_NOMEM;
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN != 0) return OPF_E_INVALID;
    opf_ctx* c = new (std::nothrow) opf_ctx();
    if (!c) return OPF_E_NOMEM;
    c->p = *p;
    c->p.r_nodes = nullptr;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<unsigned char*>(dev_workspace);
    c->ws_bytes = bytes;
    const int N = p->N, M = p->M, K = p->K, nk = 2 * K - 1;
    c->nk = nk;
    c->MU = p->mp * (M - 1) + 2;
    c->nfac = c->MU * K + M * K;
    c->gm = default_gm(p->mp);
    c->ztile = default_ztile(p->precision);

    build_grid(c, p->r_nodes);

    // FFT twiddles e^{-2 pi i t / L}
    const bool mixed = p->precision == OPF_MIXED;
    auto twiddles = [&](int L, std::vector<double>& d, std::vector<float>& f) {
        d.resize(2 * L);
        f.resize(2 * L);
        for (int t = 0; t < L; ++t) {
            const double ang = -2.0 * M_PI * t / L;
            d[2 * t] = std::cos(ang);
            d[2 * t + 1] = std::sin(ang);
            f[2 * t] = float(d[2 * t]);
            f[2 * t + 1] = float(d[2 * t + 1]);
        }
    };
    std::vector<double> twz, twt;
    std::vector<float> twz32, twt32;
    twiddles(3 * K, twz, twz32);
    twiddles(3 * M, twt, twt32);

    // carve the workspace and upload
    unsigned char* ws = c->ws;
    auto up = [&](size_t off, const void* src, size_t n) {
        return hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, c->stream);
    };
    hipError_t he = hipSuccess;
    if (he == hipSuccess) he = up(Lo.r, c->r.data(), N * 8);
    if (he == hipSuccess) he = up(Lo.rinv, c->rinv.data(), N * 8);
    if (he == hipSuccess) he = up(Lo.quad, c->quad.data(), N * 8);
    if (he == hipSuccess) he = up(Lo.d1, c->d1.data(), c->d1.size() * 8);
    if (he == hipSuccess) he = up(Lo.d2, c->d2.data(), c->d2.size() * 8);
    if (he == hipSuccess) he = up(Lo.s0, c->s0.data(), N * 4);
    // folded weights of d2/dr2 + (1/r) d/dr (the radial part of L), per parity
    std::vector<double> wl(2 * N * W9);
    for (int par = 0; par < 2; ++par)
        for (int n = 0; n < N; ++n)
            for (int j = 0; j < W9; ++j) {
                const size_t i = ((size_t)par * N + n) * W9 + j;
                wl[i] = c->d2[i] + c->rinv[n] * c->d1[i];
            }
    if (he == hipSuccess) he = up(Lo.wl, wl.data(), wl.size() * 8);
    // CFL weights: 1/dr_n (nearer neighbour; the axis mirror -r_0 for n = 0) and 1/(r_n dtheta)
    std::vector<double> cflw(2 * N);
    for (int n = 0; n < N; ++n) {
        const double left = n == 0 ? 2.0 * c->r[0] : c->r[n] - c->r[n - 1];
        const double right = n == N - 1 ? left : c->r[n + 1] - c->r[n];
        cflw[n] = 1.0 / std::min(left, right);
        cflw[N + n] = (double)p->mp * 3 * M / (2.0 * M_PI * c->r[n]);
    }
    if (he == hipSuccess) he = up(Lo.cflw, cflw.data(), cflw.size() * 8);
    if (he == hipSuccess) he = mixed ? up(Lo.twz, twz32.data(), twz32.size() * 4) : up(Lo.twz, twz.data(), twz.size() * 8);
    if (he == hipSuccess) he = mixed ? up(Lo.twt, twt32.data(), twt32.size() * 4) : up(Lo.twt, twt.data(), twt.size() * 8);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) {
        c->err = std::string("upload: ") + hipGetErrorString(he);
        delete c;
        return OPF_E_HIP;
    }
    c->t.r = reinterpret_cast<const double*>(ws + Lo.r);
    c->t.rinv = reinterpret_cast<const double*>(ws + Lo.rinv);
    c->t.quad = reinterpret_cast<const double*>(ws + Lo.quad);
    c->t.d1 = reinterpret_cast<const double*>(ws + Lo.d1);
    c->t.d2 = reinterpret_cast<const double*>(ws + Lo.d2);
    c->t.s0 = reinterpret_cast<const int*>(ws + Lo.s0);
    c->t.fac = reinterpret_cast<const double*>(ws + Lo.fac);
    c->t.img = reinterpret_cast<const double*>(ws + Lo.img);
    c->t.dinv = reinterpret_cast<const double*>(ws + Lo.dinv);
    c->t.wl = reinterpret_cast<const double*>(ws + Lo.wl);
    c->t.hom = reinterpret_cast<const double*>(ws + Lo.hom);
    c->t.ainv = reinterpret_cast<const double*>(ws + Lo.ainv);
    c->t.green = reinterpret_cast<const double*>(ws + Lo.green);
    c->t.qG_inv = c->qG_inv;
    c->twz = ws + Lo.twz;
    c->twt = ws + Lo.twt;
    c->u = reinterpret_cast<double*>(ws + Lo.u);
    c->up = reinterpret_cast<double*>(ws + Lo.up);
    c->w64 = reinterpret_cast<double*>(ws + Lo.w64);
    c->w = ws + Lo.w;
    c->Nn = ws + Lo.Nn;
    c->Np = ws + Lo.Np;
    c->H = ws + Lo.H;
    c->G = ws + Lo.G;
    c->u32 = reinterpret_cast<float*>(ws + Lo.u32);
    c->up32 = reinterpret_cast<float*>(ws + Lo.up32);
    c->beta = reinterpret_cast<double*>(ws + Lo.beta);
    c->partial = reinterpret_cast<double*>(ws + Lo.partial);
    c->dpart = reinterpret_cast<double*>(ws + Lo.dpart);
    c->cflw = reinterpret_cast<double*>(ws + Lo.cflw);
    c->cpart = reinterpret_cast<double*>(ws + Lo.cpart);
    c->wall = reinterpret_cast<double*>(ws + Lo.wall);
    // banded LU factors, influence data and Green's function on the device
    const opf_status st2 = device_tables(c, true);
    if (st2 != OPF_OK) {
        delete c;
        return st2;
    }
    *out = c;
    return OPF_OK;
}

// Forget the captured step graphs (they hold the step's arguments by value).
void drop_step_graphs(opf_ctx* c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graphs) (void)hipGraphExecDestroy(c->graphs);
    c->graph = c->graphs = nullptr;
}

opf_status opf_destroy(opf_ctx* c) {
    if (!c) return OPF_E_INVALID;
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graphs) (void)hipGraphExecDestroy(c->graphs);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    return OPF_OK;
}

opf_status opf_get_nodes(const opf_ctx* c, double* r) {
    if (!c || !r) return OPF_E_INVALID;
    std::copy(c->r.begin(), c->r.end(), r);
    return OPF_OK;
}

opf_status opf_set_state(opf_ctx* c, const void* u) {
    if (!c || !u) return OPF_E_INVALID;
    HIPCHK(c, hipMemcpyAsync(c->u, u, 3 * field_entries(c) * 16, hipMemcpyDeviceToDevice, c->stream));
    const opf_status st = refresh_derived(c);
    if (st != OPF_OK) return st;
    c->have_state = true;
    c->pc_valid = false;
    return OPF_OK;
}

opf_status opf_get_state(opf_ctx* c, void* u) {
    if (!c || !u) return OPF_E_INVALID;
    if (!c->have_state) return OPF_E_STATE;
    HIPCHK(c, hipMemcpyAsync(u, c->u, 3 * field_entries(c) * 16, hipMemcpyDeviceToDevice, c->stream));
    return OPF_OK;
}

// Steps per graph of the multi-step graph: a run of nsteps launches
// nsteps / STEP_GRAPH_STEPS of them, then single-step graphs for the rest.
constexpr int STEP_GRAPH_STEPS = 8;

// Capture `steps` consecutive steps into one executable graph.
opf_status capture_steps(opf_ctx* c, int steps, hipGraphExec_t* out) {
    if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    opf_status st = OPF_OK;
    for (int i = 0; i < steps && st == OPF_OK; ++i) st = enqueue_step(c, c->cap);
    hipError_t he = hipStreamEndCapture(c->cap, &g);
    if (st != OPF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (he != hipSuccess) {
        c->err = std::string("capture: ") + hipGetErrorString(he);
        return OPF_E_HIP;
    }
    he = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (he != hipSuccess) {
        *out = nullptr;
        c->err = std::string("instantiate: ") + hipGetErrorString(he);
        return OPF_E_HIP;
    }
    return OPF_OK;
}

opf_status opf_step(opf_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return OPF_E_INVALID;
    if (!c->have_state) return OPF_E_STATE;
    int i = 0;
    if (nsteps >= STEP_GRAPH_STEPS) {
        if (!c->graphs) {
            const opf_status st = capture_steps(c, STEP_GRAPH_STEPS, &c->graphs);
            if (st != OPF_OK) return st;
        }
        for (; i + STEP_GRAPH_STEPS <= nsteps; i += STEP_GRAPH_STEPS) HIPCHK(c, hipGraphLaunch(c->graphs, c->stream));
    }
    if (i < nsteps && !c->graph) {
        const opf_status st = capture_steps(c, 1, &c->graph);
        if (st != OPF_OK) return st;
    }
    for (; i < nsteps; ++i) HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
    if (nsteps > 0) c->pc_valid = true;
    return OPF_OK;
}

opf_status opf_profile_steps(opf_ctx* c, int32_t nsteps, double* ms, int32_t* launches) {
    if (!c || !ms || !launches || nsteps < 1) return OPF_E_INVALID;
    if (!c->have_state) return OPF_E_STATE;
    const bool mixed = c->p.precision == OPF_MIXED;
    const int nk = 5;  // zinv, theta, zfwd, solve (predictor), solve (corrector)
    // one start/stop pair per launch, recorded around the kernel itself
    std::vector<KernelTiming> ev;
    std::vector<int> kind;
    hipError_t he = hipSuccess;
    auto timing = [&](int k, KernelTiming& kt) -> hipError_t {
        hipError_t e = hipEventCreate(&kt.start);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&kt.stop);
        if (e != hipSuccess) {
            (void)hipEventDestroy(kt.start);
            return e;
        }
        ev.push_back(kt);
        kind.push_back(k);
        return hipSuccess;
    };
    const void* uin = mixed ? (const void*)c->u32 : (const void*)c->u;
    const void* upin = mixed ? (const void*)c->up32 : (const void*)c->up;
    for (int st = 0; st < nsteps && he == hipSuccess; ++st) {
        for (int half = 0; half < 2 && he == hipSuccess; ++half) {
            if (c->p.nonlinear) {
                NLArgs a = nl_args(c, half ? upin : uin, c->w, half ? c->Np : c->Nn);
                for (int stage = 0; stage < 3 && he == hipSuccess; ++stage) {
                    KernelTiming kt;
                    he = timing(stage, kt);
                    if (he == hipSuccess) he = launch_nonlinear_stage(a, c->p.precision, stage, c->stream, kt);
                }
            }
            if (he != hipSuccess) break;
            SolveArgs b = solve_args(c, half ? OPF_SOLVE_CORR : OPF_SOLVE_PRED);
            b.u0 = c->u;
            b.n0 = c->Nn;
            b.n1 = c->Np;
            b.u_out = half ? c->u : (mixed ? nullptr : c->up);
            b.u_out32 = mixed ? (half ? c->u32 : c->up32) : nullptr;
            b.w_out = c->w;
            KernelTiming kt;
            he = timing(3 + half, kt);
            if (he == hipSuccess) he = launch_solve(b, c->p.precision, c->stream, kt);
        }
    }
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    for (int k = 0; k < nk; ++k) { ms[k] = 0.0; launches[k] = 0; }
    for (size_t i = 0; i < ev.size() && he == hipSuccess; ++i) {
        float t = 0.0f;
        he = hipEventElapsedTime(&t, ev[i].start, ev[i].stop);
        ms[kind[i]] += t;
        launches[kind[i]] += 1;
    }
    for (const KernelTiming& kt : ev) {
        (void)hipEventDestroy(kt.start);
        (void)hipEventDestroy(kt.stop);
    }
    if (he != hipSuccess) {
        c->err = std::string("profile: ") + hipGetErrorString(he);
        return OPF_E_HIP;
    }
    c->pc_valid = true;
    return OPF_OK;
}

opf_status opf_vorticity(opf_ctx* c, const void* u, void* w) {
    if (!c || !u || !w) return OPF_E_INVALID;
    AuxArgs x{};
    x.N = c->p.N;
    x.M = c->p.M;
    x.K = c->p.K;
    x.nk = c->nk;
    x.mp = c->p.mp;
    x.alpha = c->p.alpha;
    x.u = static_cast<const double*>(u);
    x.w = static_cast<double*>(w);
    x.t = c->t;
    HIPCHK(c, launch_vorticity(x, c->stream));
    return OPF_OK;
}

opf_status opf_nonlinear(opf_ctx* c, const void* u, void* n) {
    if (!c || !u || !n) return OPF_E_INVALID;
    const size_t cnt = 2 * 3 * field_entries(c);
    // omega into w64, then the transforms in the working precision; the
    // 'up' / 'up32' buffers hold the input copy
    opf_status st = opf_vorticity(c, u, c->w64);
    if (st != OPF_OK) return st;
    if (c->p.precision == OPF_MIXED) {
        float* uin = c->up32;
        c->pc_valid = false;
        float* win = static_cast<float*>(c->w);
        float* nout = reinterpret_cast<float*>(c->Np);
        HIPCHK(c, to_f32(static_cast<const double*>(u), uin, cnt, c->stream));
        HIPCHK(c, to_f32(c->w64, win, cnt, c->stream));
        HIPCHK(c, launch_nonlinear(nl_args(c, uin, win, nout), OPF_MIXED, c->stream));
        HIPCHK(c, to_f64(nout, static_cast<double*>(n), cnt, c->stream));
        if (c->have_state) return refresh_derived(c);  // w was overwritten
        return OPF_OK;
    }
    HIPCHK(c, launch_nonlinear(nl_args(c, u, c->w64, n), OPF_FP64, c->stream));
    return OPF_OK;
}

opf_status opf_radial_solve(opf_ctx* c, int32_t kind, const void* rhs, void* u_out, void* p_out) {
    if (!c || !rhs || !u_out) return OPF_E_INVALID;
    if (kind != OPF_SOLVE_PRED && kind != OPF_SOLVE_CORR && kind != OPF_SOLVE_RAW) return OPF_E_INVALID;
    if (kind != OPF_SOLVE_RAW && !c->have_state) return OPF_E_STATE;
    SolveArgs a = solve_args(c, kind);
    a.u0 = c->u;
    const size_t S3 = 3 * field_entries(c);
    a.n0 = rhs;
    a.n1 = kind == OPF_SOLVE_CORR ? static_cast<const double*>(rhs) + 2 * S3 : nullptr;
    a.u_out = static_cast<double*>(u_out);
    a.p_out = static_cast<double*>(p_out);
    a.w_out = c->w64;
    // nonlinear inputs are complex128 here whatever the working precision
    HIPCHK(c, launch_solve(a, OPF_FP64, c->stream));
    return OPF_OK;
}

opf_status opf_diagnostics(opf_ctx* c, opf_diag* d) {
    if (!c || !d) return OPF_E_INVALID;
    if (!c->have_state) return OPF_E_STATE;
    const int N = c->p.N, M = c->p.M, K = c->p.K;
    AuxArgs x{};
    x.N = N;
    x.M = M;
    x.K = K;
    x.nk = c->nk;
    x.mp = c->p.mp;
    x.alpha = c->p.alpha;
    x.u = c->u;
    x.w = c->w64;
    x.partial = c->partial;
    x.wall = c->has_wall ? c->wall : nullptr;
    x.t = c->t;
    HIPCHK(c, launch_vorticity(x, c->stream));
    HIPCHK(c, launch_energy(x, c->stream));
    HIPCHK(c, launch_divg(x, c->dpart, c->stream));
    HIPCHK(c, enqueue_cfl(c));
    std::vector<double> dp(2 * (size_t)M * c->nk), cp(cfl_parts(c));
    HIPCHK(c, hipMemcpyAsync(dp.data(), c->dpart, dp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(cp.data(), c->cpart, cp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> part(2 * M), uz(2 * N);
    double beta = 0.0;
    const size_t S = field_entries(c);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, 2 * M * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(uz.data(), c->u + 2 * (2 * S + (size_t)(K - 1) * N), 2 * N * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&beta, c->beta, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double su = 0.0, sw = 0.0;
    for (int m = 0; m < M; ++m) {
        const double cm = m == 0 ? 1.0 : 2.0;
        su += cm * part[2 * m];
        sw += cm * part[2 * m + 1];
    }
    const double lz = 2.0 * M_PI / c->p.alpha;
    const double vol = 2.0 * M_PI * lz / c->p.mp;
    double flux = 0.0, dz = 0.0;
    for (int n = 0; n < N; ++n) flux += c->quad[n] * uz[2 * n];
    for (int j = 0; j < W9; ++j) dz += c->d1[(N - 1) * W9 + j] * uz[2 * (c->s0[N - 1] + j)];
    *d = opf_diag{};
    d->E = 0.5 * vol * su;
    d->D = vol * sw / c->p.Re;
    d->flux = flux;
    d->beta = beta;
    d->I = 4.0 / c->p.Re * (1.0 + beta) * vol * flux;
    d->tau_w = -dz;
    d->E_lam = M_PI * lz / (6.0 * c->p.mp);
    d->I_lam = d->D_lam = 2.0 * M_PI * lz / (c->p.mp * c->p.Re);
    for (size_t q = 0; q < dp.size() / 2; ++q) {
        d->g_norm = std::max(d->g_norm, dp[2 * q]);
        d->div_max = std::max(d->div_max, dp[2 * q + 1]);
    }
    double cm = 0.0;
    for (double v : cp) cm = std::max(cm, v);
    d->cfl = c->p.dt * cm;
    if (!std::isfinite(d->E) || !std::isfinite(d->D) || !std::isfinite(d->cfl)) return OPF_E_NUMERIC;
    if (d->cfl > 1.0) {
        c->err = "CFL number above 1";
        return OPF_E_NUMERIC;
    }
    return OPF_OK;
}

opf_status opf_set_dt(opf_ctx* c, double dt) {
    if (!c || !(dt > 0) || !std::isfinite(dt)) return OPF_E_INVALID;
    if (c->in_ensemble) {
        c->err = "ensemble members keep the dt of their class graph";
        return OPF_E_UNSUPPORTED;
    }
    if (dt == c->p.dt) return OPF_OK;
    const double old = c->p.dt;
    c->p.dt = dt;
    // stream order puts the rebuild after every step already enqueued
    const opf_status st = device_tables(c, false);
    if (st != OPF_OK) {
        const std::string why = c->err;
        c->p.dt = old;
        const opf_status back = device_tables(c, false);
        c->err = why;
        if (back != OPF_OK) c->have_state = false;  // tables lost: refuse to step
        return st;
    }
    drop_step_graphs(c);
    return OPF_OK;
}

opf_status opf_set_wall_velocity(opf_ctx* c, const double* b) {
    if (!c) return OPF_E_INVALID;
    if (c->in_ensemble) {
        c->err = "ensemble members keep a no-slip wall";
        return OPF_E_UNSUPPORTED;
    }
    const int M = c->p.M, K = c->p.K, nk = c->nk;
    if (b) {
        const size_t n = (size_t)3 * M * nk * 2;
        std::vector<double> w(b, b + n);
        auto at = [&](int comp, int mi, int kk) { return &w[(((size_t)comp * M + mi) * nk + kk) * 2]; };
        for (int comp = 0; comp < 3; ++comp) {
            for (size_t i = 0; i < n / 3; ++i)
                if (!std::isfinite(w[comp * (n / 3) + i])) return OPF_E_INVALID;
            at(comp, 0, K - 1)[1] = 0.0;  // (0,0) of a real field
            for (int kp = 1; kp < K; ++kp) {  // m = 0, k < 0: conjugates of k > 0
                at(comp, 0, K - 1 - kp)[0] = at(comp, 0, K - 1 + kp)[0];
                at(comp, 0, K - 1 - kp)[1] = -at(comp, 0, K - 1 + kp)[1];
            }
        }
        if (at(0, 0, K - 1)[0] != 0.0) {
            c->err = "the (0,0) radial wall velocity (net flux through the wall) must be zero";
            return OPF_E_INVALID;
        }
        HIPCHK(c, hipMemcpyAsync(c->wall, w.data(), n * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->has_wall = b != nullptr;
    drop_step_graphs(c);  // the step graph holds the previous boundary condition
    return OPF_OK;
}

opf_status opf_set_rotation(opf_ctx* c, double ox, double oy, double oz) {
    if (!c || !std::isfinite(ox) || !std::isfinite(oy) || !std::isfinite(oz)) return OPF_E_INVALID;
    if (c->in_ensemble || !c->p.nonlinear || ((ox != 0.0 || oy != 0.0) && c->p.mp != 1)) {
        c->err = c->in_ensemble ? "ensemble members step without forcing"
                 : !c->p.nonlinear ? "the force is added to the nonlinear term, which is switched off"
                                   : "a transverse rotation axis couples m to m +- 1 and needs mp = 1";
        return OPF_E_UNSUPPORTED;
    }
    c->rot[0] = ox;
    c->rot[1] = oy;
    c->rot[2] = oz;
    drop_step_graphs(c);  // the step graph holds the previous value
    return OPF_OK;
}

opf_status opf_pc_difference(opf_ctx* c, double* out) {
    if (!c || !out) return OPF_E_INVALID;
    if (!c->have_state || !c->pc_valid) return OPF_E_STATE;
    HIPCHK(c, enqueue_pcdiff(c));
    std::vector<double> part(c->p.M);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *out = weighted_norm(part);
    return std::isfinite(*out) ? OPF_OK : OPF_E_NUMERIC;
}

opf_status opf_step_adaptive(opf_ctx* c, int32_t nsteps, const opf_dt_control* k, double* trace,
                             opf_dt_report* rep) {
    if (!c || !k || !rep || nsteps < 0) return OPF_E_INVALID;
    *rep = opf_dt_report{};
    rep->dt = c->p.dt;
    if (c->in_ensemble) {
        c->err = "ensemble members keep the dt of their class graph";
        return OPF_E_UNSUPPORTED;
    }
    if (!(k->courant > 0) || !(k->pc_tol >= 0) || !(k->dt_min > 0) || !(k->dt_max >= k->dt_min) ||
        !(k->grow >= 0) || k->check_every < 1 || !std::isfinite(k->dt_max) || !std::isfinite(k->grow))
        return OPF_E_INVALID;
    if (c->p.dt < k->dt_min || c->p.dt > k->dt_max) {
        c->err = "dt outside [dt_min, dt_max]";
        return OPF_E_INVALID;
    }
    if (!c->have_state) return OPF_E_STATE;
    const int M = c->p.M;
    std::vector<double> part(M), cp(cfl_parts(c));
    int done = 0;
    while (done < nsteps) {
        const int run = std::min(nsteps - done, k->check_every - done % k->check_every);
        for (int i = 0; i < run; ++i) {
            if (trace) trace[done + i] = c->p.dt;
            rep->t += c->p.dt;
        }
        const opf_status st = opf_step(c, run);
        if (st != OPF_OK) return st;
        done += run;
        rep->steps = done;
        if (done % k->check_every != 0) break;  // only at the end of the run
        HIPCHK(c, enqueue_cfl(c));
        HIPCHK(c, enqueue_pcdiff(c));
        HIPCHK(c, hipMemcpyAsync(cp.data(), c->cpart, cp.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, M * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double cm = 0.0;
        for (double v : cp) cm = std::max(cm, v);
        const double dt = c->p.dt;
        rep->cfl = dt * cm;
        rep->pc_diff = weighted_norm(part);
        rep->checks += 1;
        if (!std::isfinite(rep->cfl) || !std::isfinite(rep->pc_diff)) {
            c->err = "non-finite CFL number or correction";
            return OPF_E_NUMERIC;
        }
        const double nw = next_dt(dt, rep->cfl, rep->pc_diff, *k);
        if (nw < k->dt_min) {
            c->err = "time step below dt_min";
            return OPF_E_NUMERIC;
        }
        if (nw != dt) {
            const auto t0 = std::chrono::steady_clock::now();
            const opf_status s2 = opf_set_dt(c, nw);
            rep->rebuild_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (s2 != OPF_OK) return s2;
            rep->changes += 1;
            rep->dt = nw;
        }
    }
    rep->dt = c->p.dt;
    return OPF_OK;
}

opf_status opf_vec_dot(opf_ctx* c, const void* a, const void* b, double* out) {
    if (!c || !a || !b || !out) return OPF_E_INVALID;
    const int M = c->p.M;
    hipLaunchKernelGGL(k_wdot, dim3(M), dim3(256), 0, c->stream, static_cast<const double*>(a),
                       static_cast<const double*>(b), c->t.quad, c->partial, c->p.N, M, c->nk);
    HIPCHK(c, hipGetLastError());
    std::vector<double> part(M);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, M * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += (m == 0 ? 1.0 : 2.0) * part[m];
    *out = s;
    return std::isfinite(s) ? OPF_OK : OPF_E_NUMERIC;
}

opf_status opf_vec_axpby(opf_ctx* c, double a, const void* x, double b, void* y) {
    if (!c || !x || !y) return OPF_E_INVALID;
    const size_t n = 2 * 3 * field_entries(c);
    hipLaunchKernelGGL(k_axpby, dim3((n + 255) / 256), dim3(256), 0, c->stream, a,
                       static_cast<const double*>(x), b, static_cast<double*>(y), n);
    HIPCHK(c, hipGetLastError());
    return OPF_OK;
}

opf_status opf_newton_residual(opf_ctx* c, const void* x, double T, double shift, void* F, double* norm) {
    if (!c || !x || !F) return OPF_E_INVALID;
    if (!(T >= 0)) return OPF_E_INVALID;
    const int nsteps = (int)std::lround(T / c->p.dt);
    opf_status st = opf_set_state(c, x);
    if (st != OPF_OK) return st;
    st = opf_step(c, nsteps);
    if (st != OPF_OK) return st;
    const size_t total = 3 * field_entries(c);
    hipLaunchKernelGGL(k_shift_sub, dim3((total + 255) / 256), dim3(256), 0, c->stream, c->u,
                       static_cast<const double*>(x), static_cast<double*>(F), c->p.N, c->nk, c->p.K, total,
                       c->p.alpha, shift);
    HIPCHK(c, hipGetLastError());
    if (norm) {
        double s2 = 0.0;
        st = opf_vec_dot(c, F, F, &s2);
        if (st != OPF_OK) return st;
        *norm = std::sqrt(std::max(s2, 0.0));
    }
    return OPF_OK;
}

namespace {
// ||F|| at a trial point of a Newton step.  A trial state the time step
// cannot follow (the explicit terms past their stability limit) gives a
// non-finite norm: that trial counts as +infinity, i.e. rejected, and the
// caller shortens the step.
opf_status trial_residual(opf_ctx* c, const void* x, double T, double shift, void* F, double* norm) {
    const opf_status st = opf_newton_residual(c, x, T, shift, F, norm);
    if (st == OPF_E_NUMERIC) {
        *norm = INFINITY;
        return OPF_OK;
    }
    return st;
}
}  // namespace

opf_status opf_hookstep_solve(const double* hb, int32_t k, double beta, double delta, double* y, double* mu_out,
                              double* resid) {
    if (!hb || !y || !mu_out || !resid || k < 1 || !(beta >= 0) || !(delta > 0)) return OPF_E_INVALID;
    const int rows = k + 1;
    // one-sided Jacobi SVD: rotate the columns of A = Hb until they are
    // orthogonal; A W = U S, W the accumulated rotations
    std::vector<double> A(hb, hb + (size_t)rows * k), W((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) W[(size_t)j * k + j] = 1.0;
    auto col = [&](std::vector<double>& M, int nr, int nc, int i, int j) -> double& { return M[(size_t)i * nc + j]; };
    for (int sweep = 0; sweep < 80; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                double a = 0.0, b = 0.0, g = 0.0;
                for (int i = 0; i < rows; ++i) {
                    const double x = col(A, rows, k, i, p), z = col(A, rows, k, i, q);
                    a += x * x;
                    b += z * z;
                    g += x * z;
                }
                if (g == 0.0 || std::fabs(g) <= 1e-15 * std::sqrt(a * b)) continue;
                rotated = true;
                const double zeta = (b - a) / (2.0 * g);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < rows; ++i) {
                    const double x = col(A, rows, k, i, p), z = col(A, rows, k, i, q);
                    col(A, rows, k, i, p) = cs * x - sn * z;
                    col(A, rows, k, i, q) = sn * x + cs * z;
                }
                for (int i = 0; i < k; ++i) {
                    const double x = col(W, k, k, i, p), z = col(W, k, k, i, q);
                    col(W, k, k, i, p) = cs * x - sn * z;
                    col(W, k, k, i, q) = sn * x + cs * z;
                }
            }
        if (!rotated) break;
    }
    std::vector<double> sv(k), pv(k);
    double smax = 0.0;
    for (int j = 0; j < k; ++j) {
        double s2 = 0.0;
        for (int i = 0; i < rows; ++i) s2 += col(A, rows, k, i, j) * col(A, rows, k, i, j);
        sv[j] = std::sqrt(s2);
        smax = std::max(smax, sv[j]);
    }
    for (int j = 0; j < k; ++j) {
        if (!(sv[j] > 1e-14 * smax)) sv[j] = 0.0;
        pv[j] = sv[j] > 0 ? beta * col(A, rows, k, 0, j) / sv[j] : 0.0;  // beta u_j[0]
    }
    auto zlen = [&](double mu, double* dsum) {
        double l2 = 0.0, d = 0.0;
        for (int j = 0; j < k; ++j) {
            if (sv[j] == 0.0) continue;
            const double den = sv[j] * sv[j] + mu, z = pv[j] * sv[j] / den;
            l2 += z * z;
            d += z * z / den;
        }
        if (dsum) *dsum = d;
        return std::sqrt(l2);
    };
    double mu = 0.0;
    if (zlen(0.0, nullptr) > delta) {
        // ||z(mu)|| decreases from above delta at 0 to 0: bracket, then Newton
        // on 1/||z|| - 1/delta, falling back to bisection
        double lo = 0.0, hi = 1.0;
        double pmax = 0.0;
        for (int j = 0; j < k; ++j) pmax = std::max(pmax, std::fabs(pv[j]) * sv[j]);
        hi = std::max(pmax * std::sqrt((double)k) / delta, 1e-300);
        while (zlen(hi, nullptr) > delta) hi *= 2.0;
        mu = 0.5 * (lo + hi);
        for (int it = 0; it < 300; ++it) {
            double d = 0.0;
            const double L = zlen(mu, &d);
            if (L > delta) lo = mu;
            else hi = mu;
            if (std::fabs(L - delta) <= 4e-16 * delta || hi - lo <= 4e-16 * hi) break;
            // d||z||/dmu = -d / ||z||; Newton step on 1/||z|| - 1/delta
            double next = d > 0 ? mu + (1.0 / delta - 1.0 / L) * L * L * L / d : -1.0;
            if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
            mu = next;
        }
    }
    for (int i = 0; i < k; ++i) y[i] = 0.0;
    for (int j = 0; j < k; ++j) {
        if (sv[j] == 0.0) continue;
        const double z = pv[j] * sv[j] / (sv[j] * sv[j] + mu);
        for (int i = 0; i < k; ++i) y[i] += col(W, k, k, i, j) * z;
    }
    double r2 = 0.0;
    for (int i = 0; i < rows; ++i) {
        double acc = i == 0 ? beta : 0.0;
        for (int j = 0; j < k; ++j) acc -= hb[(size_t)i * k + j] * y[j];
        r2 += acc * acc;
    }
    *mu_out = mu;
    *resid = std::sqrt(r2);
    return std::isfinite(*resid) ? OPF_OK : OPF_E_NUMERIC;
}

opf_status opf_shoot_workspace_size(const opf_ctx* c, int32_t S, int32_t m, size_t* bytes) {
    if (!c || !bytes || S < 1 || m < 1) return OPF_E_INVALID;
    *bytes = ((size_t)(m + 6) * S + 3) * 3 * field_entries(c) * 16;
    return OPF_OK;
}

opf_status opf_shoot_solve(opf_ctx* c, void* x_dev, double* T_io, double* s_io, const opf_shoot_opts* o,
                           void* work, size_t work_bytes, opf_shoot_report* rep) {
    if (!c || !x_dev || !T_io || !s_io || !o || !work || !rep) return OPF_E_INVALID;
    const int S = o->sections, n = o->steps, m = o->gmres_m;
    if (S < 1 || n < 1 || m < 1 || o->max_newton < 0 || !(*T_io > 0) || !std::isfinite(*s_io) ||
        !(o->fd_eps > 0) || !(o->tol >= 0) || !(o->gmres_tol >= 0))
        return OPF_E_INVALID;
    size_t need = 0;
    if (opf_shoot_workspace_size(c, S, m, &need) != OPF_OK || work_bytes < need) return OPF_E_NOMEM;
    if (c->in_ensemble) {
        c->err = "ensemble members keep the dt of their class graph";
        return OPF_E_UNSUPPORTED;
    }
    *rep = opf_shoot_report{};
    const double dt0 = c->p.dt;
    const size_t total = 3 * field_entries(c), vb = total * 16, eb = (size_t)S * vb;
    unsigned char* base = static_cast<unsigned char*>(work);
    // extended vectors: S fields on the device, (T, s) entries on the host
    const int nvec = m + 6;
    auto ev = [&](int i) { return base + (size_t)i * eb; };
    auto fld = [&](unsigned char* e, int sec) { return static_cast<void*>(e + (size_t)sec * vb); };
    std::vector<double> sc(2 * (size_t)nvec, 0.0);  // host (T, s) entries per extended vector
    const int iG0 = m + 1, iW = m + 2, iGt = m + 3, iXe = m + 4, iGe = m + 5;
    unsigned char* extra = base + (size_t)nvec * eb;
    void* phT = extra;           // xdot_1
    void* phS = extra + vb;      // d_z x_1
    void* tmp = extra + 2 * vb;  // scratch field
    unsigned char* X = static_cast<unsigned char*>(x_dev);
    double XT = *T_io, Xs = *s_io;
    const int max_hook = o->max_hook > 0 ? o->max_hook : 12;
    const double delta_max = o->tr_delta_max > 0 ? o->tr_delta_max : INFINITY;
    double delta = o->tr_delta0;
#define SHCHK(call)                    \
    do {                               \
        const opf_status st_ = (call); \
        if (st_ != OPF_OK) {           \
            (void)opf_set_dt(c, dt0);  \
            return st_;                \
        }                              \
    } while (0)
    // <A, B> over the sections plus the scalar entries (a, b: host pairs)
    auto xdot = [&](unsigned char* A, const double* a, unsigned char* B, const double* b, double* out) -> opf_status {
        double acc = a[0] * b[0] + a[1] * b[1];
        for (int i = 0; i < S; ++i) {
            double d = 0.0;
            const opf_status st = opf_vec_dot(c, fld(A, i), fld(B, i), &d);
            if (st != OPF_OK) return st;
            acc += d;
        }
        *out = acc;
        return OPF_OK;
    };
    // Y = a A + b Y
    auto xaxpby = [&](double a, unsigned char* A, const double* as, double b, unsigned char* Y, double* ys) {
        for (int i = 0; i < S; ++i) {
            const opf_status st = opf_vec_axpby(c, a, fld(A, i), b, fld(Y, i));
            if (st != OPF_OK) return st;
        }
        ys[0] = a * as[0] + b * ys[0];
        ys[1] = a * as[1] + b * ys[1];
        return OPF_OK;
    };
    auto set_T = [&](double T) -> opf_status { return opf_set_dt(c, T / ((double)S * n)); };
    // G(Y) into Gout (scalar entries 0)
    auto residual = [&](unsigned char* Y, const double* ys, unsigned char* Gout, double* gs) -> opf_status {
        opf_status st = set_T(ys[0]);
        if (st != OPF_OK) return st;
        for (int i = 0; i < S; ++i) {
            if ((st = opf_set_state(c, fld(Y, i))) != OPF_OK) return st;
            if ((st = opf_step(c, n)) != OPF_OK) return st;
            const void* next = fld(Y, i + 1 < S ? i + 1 : 0);
            hipLaunchKernelGGL(k_shift_sub, dim3((total + 255) / 256), dim3(256), 0, c->stream, c->u,
                               static_cast<const double*>(next), static_cast<double*>(fld(Gout, i)), c->p.N, c->nk,
                               c->p.K, total, c->p.alpha, i + 1 < S ? 0.0 : ys[1]);
            HIPCHK(c, hipGetLastError());
        }
        gs[0] = gs[1] = 0.0;
        rep->residual_evals += 1;
        return OPF_OK;
    };
    auto nrm = [&](unsigned char* A, const double* a, double* out) -> opf_status {
        double d = 0.0;
        const opf_status st = xdot(A, a, A, a, &d);
        *out = std::sqrt(std::max(d, 0.0));
        return st;
    };
    // copy the guess into W, evaluate G0
    double* sW = &sc[2 * iW];
    HIPCHK(c, hipMemcpyAsync(ev(iW), X, eb, hipMemcpyDeviceToDevice, c->stream));
    sW[0] = XT;
    sW[1] = Xs;
    double* sG0 = &sc[2 * iG0];
    SHCHK(residual(ev(iW), sW, ev(iG0), sG0));
    double fn = 0.0, xn = 0.0;
    SHCHK(nrm(ev(iG0), sG0, &fn));
    SHCHK(nrm(ev(iW), sW, &xn));
    rep->residual_history[0] = rep->residual = fn / xn;
    int it = 0;
    for (; it < o->max_newton && rep->residual > o->tol; ++it) {
        // phase vectors at x_1 and T
        if (o->free_T) {
            SHCHK(set_T(sW[0]));
            SHCHK(opf_set_state(c, fld(ev(iW), 0)));
            SHCHK(opf_step(c, 1));
            HIPCHK(c, hipMemcpyAsync(phT, c->u, vb, hipMemcpyDeviceToDevice, c->stream));
            SHCHK(opf_vec_axpby(c, -1.0 / c->p.dt, fld(ev(iW), 0), 1.0 / c->p.dt, phT));
        }
        if (o->free_s) {
            hipLaunchKernelGGL(k_ddz, dim3((total + 255) / 256), dim3(256), 0, c->stream,
                               static_cast<const double*>(fld(ev(iW), 0)), static_cast<double*>(phS), c->p.N, c->nk,
                               c->p.K, total, c->p.alpha);
            HIPCHK(c, hipGetLastError());
        }
        // J V into extended vector `out` (V has unit norm)
        auto jv = [&](int iv, int iout) -> opf_status {
            double* sv = &sc[2 * iv];
            if (!o->free_T) sv[0] = 0.0;
            if (!o->free_s) sv[1] = 0.0;
            double vn = 0.0;
            opf_status st = nrm(ev(iv), sv, &vn);
            if (st != OPF_OK) return st;
            double* so = &sc[2 * iout];
            if (!(vn > 0)) {
                for (int i = 0; i < S; ++i)
                    if ((st = opf_vec_axpby(c, 0.0, fld(ev(iv), i), 0.0, fld(ev(iout), i))) != OPF_OK) return st;
                so[0] = so[1] = 0.0;
                return OPF_OK;
            }
            const double eps = o->fd_eps * std::max(xn, 1.0) / vn;
            double* sXe = &sc[2 * iXe];
            double* sGe = &sc[2 * iGe];
            HIPCHK(c, hipMemcpyAsync(ev(iXe), ev(iW), eb, hipMemcpyDeviceToDevice, c->stream));
            sXe[0] = sW[0];
            sXe[1] = sW[1];
            if ((st = xaxpby(eps, ev(iv), sv, 1.0, ev(iXe), sXe)) != OPF_OK) return st;
            if ((st = residual(ev(iXe), sXe, ev(iGe), sGe)) != OPF_OK) return st;
            HIPCHK(c, hipMemcpyAsync(ev(iout), ev(iGe), eb, hipMemcpyDeviceToDevice, c->stream));
            so[0] = so[1] = 0.0;
            if ((st = xaxpby(-1.0 / eps, ev(iG0), sG0, 1.0 / eps, ev(iout), so)) != OPF_OK) return st;
            so[0] = so[1] = 0.0;
            if (o->free_T && (st = opf_vec_dot(c, phT, fld(ev(iv), 0), &so[0])) != OPF_OK) return st;
            if (o->free_s && (st = opf_vec_dot(c, phS, fld(ev(iv), 0), &so[1])) != OPF_OK) return st;
            rep->products += 1;
            return OPF_OK;
        };
        // Arnoldi from v_1 = -G / ||G||
        {
            double* s0v = &sc[0];
            s0v[0] = s0v[1] = 0.0;
            for (int i = 0; i < S; ++i) SHCHK(opf_vec_axpby(c, -1.0 / fn, fld(ev(iG0), i), 0.0, fld(ev(0), i)));
            s0v[0] = -sG0[0] / fn;
            s0v[1] = -sG0[1] / fn;
        }
        std::vector<double> Hr((size_t)(m + 1) * m, 0.0), Hw((size_t)(m + 1) * m, 0.0);
        std::vector<double> cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
        g[0] = fn;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            SHCHK(jv(j, j + 1));
            for (int i = 0; i <= j; ++i) {
                double h = 0.0;
                SHCHK(xdot(ev(j + 1), &sc[2 * (j + 1)], ev(i), &sc[2 * i], &h));
                Hr[(size_t)i * m + j] = h;
                SHCHK(xaxpby(-h, ev(i), &sc[2 * i], 1.0, ev(j + 1), &sc[2 * (j + 1)]));
            }
            double hn = 0.0;
            SHCHK(nrm(ev(j + 1), &sc[2 * (j + 1)], &hn));
            Hr[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i <= j + 1; ++i) Hw[(size_t)i * m + j] = Hr[(size_t)i * m + j];
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Hw[(size_t)i * m + j] + sn[i] * Hw[(size_t)(i + 1) * m + j];
                Hw[(size_t)(i + 1) * m + j] = -sn[i] * Hw[(size_t)i * m + j] + cs[i] * Hw[(size_t)(i + 1) * m + j];
                Hw[(size_t)i * m + j] = t;
            }
            const double d = std::hypot(Hw[(size_t)j * m + j], hn);
            cs[j] = d == 0.0 ? 1.0 : Hw[(size_t)j * m + j] / d;
            sn[j] = d == 0.0 ? 0.0 : hn / d;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            if (std::fabs(g[k]) <= o->gmres_tol * fn || hn == 0.0) break;
            SHCHK(xaxpby(1.0 / hn, ev(j + 1), &sc[2 * (j + 1)], 0.0, ev(j + 1), &sc[2 * (j + 1)]));
        }
        std::vector<double> hb((size_t)(k + 1) * k), y(k);
        for (int i = 0; i <= k; ++i)
            for (int j = 0; j < k; ++j) hb[(size_t)i * k + j] = Hr[(size_t)i * m + j];
        double mu = 0.0, r = 0.0;
        if (!(delta > 0)) {
            SHCHK(opf_hookstep_solve(hb.data(), k, fn, INFINITY, y.data(), &mu, &r));
            double l2 = 0.0;
            for (double v : y) l2 += v * v;
            delta = std::sqrt(l2);
        }
        // trial X + dx in Xe, its residual in Gt
        bool accepted = false;
        double fnew = 0.0;
        double* sXe = &sc[2 * iXe];
        double* sGt = &sc[2 * iGt];
        for (int trial = 0; trial < max_hook; ++trial) {
            SHCHK(opf_hookstep_solve(hb.data(), k, fn, delta, y.data(), &mu, &r));
            double dn2 = 0.0;
            for (double v : y) dn2 += v * v;
            const double dn = std::sqrt(dn2);
            HIPCHK(c, hipMemcpyAsync(ev(iXe), ev(iW), eb, hipMemcpyDeviceToDevice, c->stream));
            sXe[0] = sW[0];
            sXe[1] = sW[1];
            for (int i = 0; i < k; ++i) SHCHK(xaxpby(y[i], ev(i), &sc[2 * i], 1.0, ev(iXe), sXe));
            SHCHK(residual(ev(iXe), sXe, ev(iGt), sGt));
            {  // a trial the time step cannot follow (non-finite norm) is rejected
                const opf_status st = nrm(ev(iGt), sGt, &fnew);
                if (st == OPF_E_NUMERIC) fnew = INFINITY;
                else SHCHK(st);
            }
            rep->hook_trials += 1;
            const double den = fn * fn - r * r;
            const double rho = den > 0 ? (fn * fn - fnew * fnew) / den : -INFINITY;
            if (rho >= 0.1) {
                accepted = true;
                if (rho > 0.75 && dn >= 0.99 * delta) delta = std::min(2.0 * delta, delta_max);
                else if (rho < 0.25) delta = 0.5 * dn;
                break;
            }
            delta = 0.5 * dn;
        }
        rep->tr_delta = delta;
        if (!accepted) {
            rep->stalled = 1;
            break;
        }
        HIPCHK(c, hipMemcpyAsync(ev(iW), ev(iXe), eb, hipMemcpyDeviceToDevice, c->stream));
        sW[0] = sXe[0];
        sW[1] = sXe[1];
        HIPCHK(c, hipMemcpyAsync(ev(iG0), ev(iGt), eb, hipMemcpyDeviceToDevice, c->stream));
        sG0[0] = sGt[0];
        sG0[1] = sGt[1];
        fn = fnew;
        SHCHK(nrm(ev(iW), sW, &xn));
        rep->residual = fn / xn;
        if (it + 1 < 32) rep->residual_history[it + 1] = rep->residual;
    }
#undef SHCHK
    HIPCHK(c, hipMemcpyAsync(X, ev(iW), eb, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *T_io = sW[0];
    *s_io = sW[1];
    rep->T = sW[0];
    rep->shift = sW[1];
    rep->newton_iterations = it;
    rep->converged = rep->residual <= o->tol ? 1 : 0;
    return opf_set_dt(c, dt0);
}

opf_status opf_hessenberg_eigvals(const double* h, int32_t k, double* re, double* im) {
    if (!h || !re || !im || k < 1) return OPF_E_INVALID;
    std::vector<double> A((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
        for (int j = std::max(0, i - 1); j < k; ++j) A[(size_t)i * k + j] = h[(size_t)i * k + j];
    auto a = [&](int i, int j) -> double& { return A[(size_t)i * k + j]; };
    std::vector<std::pair<double, double>> ev;
    const double eps = std::ldexp(1.0, -52);
    int n = k - 1, iter = 0, total = 0;
    while (n >= 0) {
        // deflate at the lowest negligible subdiagonal entry of the active block
        int l = n;
        for (; l > 0; --l) {
            const double s0 = std::fabs(a(l - 1, l - 1)) + std::fabs(a(l, l));
            if (std::fabs(a(l, l - 1)) <= eps * (s0 > 0 ? s0 : 1.0)) {
                a(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == n) {  // 1 x 1 block
            ev.push_back({a(n, n), 0.0});
            n -= 1;
            iter = 0;
            continue;
        }
        if (l == n - 1) {  // 2 x 2 block in closed form
            const double p = a(n - 1, n - 1), q = a(n - 1, n), r = a(n, n - 1), d = a(n, n);
            const double half = 0.5 * (p - d), disc = half * half + q * r;
            if (disc >= 0) {
                const double z = half + (half >= 0 ? 1.0 : -1.0) * std::sqrt(disc);
                const double l1 = d + z, l2 = z != 0.0 ? d - q * r / z : d;
                ev.push_back({l1, 0.0});
                ev.push_back({l2, 0.0});
            } else {
                const double w = std::sqrt(-disc);
                ev.push_back({d + half, w});
                ev.push_back({d + half, -w});
            }
            n -= 2;
            iter = 0;
            continue;
        }
        if (++total > 60 * k) return OPF_E_NUMERIC;
        ++iter;
        // double shift: the eigenvalues of the trailing 2 x 2 block, or an
        // exceptional shift every 10 stalled steps
        double sh = a(n - 1, n - 1) + a(n, n);
        double tq = a(n - 1, n - 1) * a(n, n) - a(n - 1, n) * a(n, n - 1);
        if (iter % 10 == 0) {
            const double x0 = std::fabs(a(n, n - 1)) + std::fabs(a(n - 1, n - 2));
            sh = 1.5 * x0;
            tq = x0 * x0;
        }
        double x = a(l, l) * a(l, l) + a(l, l + 1) * a(l + 1, l) - sh * a(l, l) + tq;
        double y = a(l + 1, l) * (a(l, l) + a(l + 1, l + 1) - sh);
        double z = a(l + 1, l) * a(l + 2, l + 1);
        for (int q = l; q <= n - 1; ++q) {
            const int nr = q < n - 1 ? 3 : 2;  // reflector size
            double v[3] = {x, y, nr == 3 ? z : 0.0};
            const double nv = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (nv > 0.0) {
                v[0] += v[0] >= 0 ? nv : -nv;
                const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                // left: rows q..q+nr-1, columns of the active block
                for (int j = std::max(l, q - 1); j <= n; ++j) {
                    double dot = 0.0;
                    for (int t = 0; t < nr; ++t) dot += v[t] * a(q + t, j);
                    const double f = 2.0 * dot / vv;
                    for (int t = 0; t < nr; ++t) a(q + t, j) -= f * v[t];
                }
                // right: columns q..q+nr-1, rows of the active block
                for (int i = l; i <= std::min(n, q + 3); ++i) {
                    double dot = 0.0;
                    for (int t = 0; t < nr; ++t) dot += a(i, q + t) * v[t];
                    const double f = 2.0 * dot / vv;
                    for (int t = 0; t < nr; ++t) a(i, q + t) -= f * v[t];
                }
            }
            if (q < n - 1) {
                x = a(q + 1, q);
                y = a(q + 2, q);
                if (q < n - 2) z = a(q + 3, q);
            }
        }
        // restore exact zeros below the subdiagonal of the active block
        for (int i = l + 2; i <= n; ++i)
            for (int j = l; j < i - 1; ++j) a(i, j) = 0.0;
    }
    std::stable_sort(ev.begin(), ev.end(), [](const std::pair<double, double>& p, const std::pair<double, double>& q) {
        const double mp = std::hypot(p.first, p.second), mq = std::hypot(q.first, q.second);
        if (mp != mq) return mp > mq;
        return p.second > q.second;
    });
    for (int i = 0; i < k; ++i) {
        re[i] = ev[i].first;
        im[i] = ev[i].second;
    }
    return OPF_OK;
}

opf_status opf_arnoldi_workspace_size(const opf_ctx* c, int32_t m, size_t* bytes) {
    if (!c || !bytes || m < 1) return OPF_E_INVALID;
    *bytes = (size_t)(m + 4) * 3 * field_entries(c) * 16;
    return OPF_OK;
}

opf_status opf_arnoldi(opf_ctx* c, const void* x_dev, double T, double shift, const void* v0, int32_t m,
                       int32_t nev, double tol, int32_t check_every, double fd_eps, void* work, size_t work_bytes,
                       double* ritz_re, double* ritz_im, double* hess, opf_arnoldi_report* rep) {
    if (!c || !x_dev || !v0 || !work || !ritz_re || !ritz_im || !rep || m < 1 || nev < 1 || nev > m ||
        check_every < 1 || !(tol >= 0) || !(fd_eps > 0))
        return OPF_E_INVALID;
    size_t need = 0;
    if (opf_arnoldi_workspace_size(c, m, &need) != OPF_OK || work_bytes < need) return OPF_E_NOMEM;
    *rep = opf_arnoldi_report{};
    const size_t vb = 3 * field_entries(c) * 16;
    unsigned char* base = static_cast<unsigned char*>(work);
    auto vec = [&](int i) { return static_cast<void*>(base + (size_t)i * vb); };
    void* P0 = vec(m + 1);   // P(x) = shift(Phi_T(x), -s)
    void* xe = vec(m + 2);   // x + eps v
    void* Fe = vec(m + 3);   // F(x + eps v)
    const void* x = x_dev;
    auto nrm = [&](const void* v, double* out) {
        double s2 = 0.0;
        const opf_status st = opf_vec_dot(c, v, v, &s2);
        *out = std::sqrt(std::max(s2, 0.0));
        return st;
    };
#define ARCHK(call)                    \
    do {                               \
        const opf_status st_ = (call); \
        if (st_ != OPF_OK) return st_; \
    } while (0)
    double xn = 0.0, vn = 0.0;
    ARCHK(opf_newton_residual(c, x, T, shift, P0, nullptr));
    ARCHK(opf_vec_axpby(c, 1.0, x, 1.0, P0));
    ARCHK(nrm(x, &xn));
    xn = std::max(xn, 1.0);
    ARCHK(nrm(v0, &vn));
    if (!(vn > 0)) return OPF_E_INVALID;
    ARCHK(opf_vec_axpby(c, 1.0 / vn, v0, 0.0, vec(0)));
    std::vector<double> H((size_t)(m + 1) * m, 0.0), prev, cur(2 * (size_t)m);
    bool have_prev = false;
    for (int j = 0; j < m; ++j) {
        // J v_j into v_{j+1}: (F(x + eps v) + (x + eps v) - P(x)) / eps, ||v_j|| = 1
        const double eps = fd_eps * xn;
        ARCHK(opf_vec_axpby(c, 1.0, x, 0.0, xe));
        ARCHK(opf_vec_axpby(c, eps, vec(j), 1.0, xe));
        ARCHK(opf_newton_residual(c, xe, T, shift, Fe, nullptr));
        ARCHK(opf_vec_axpby(c, 1.0, Fe, 0.0, vec(j + 1)));
        ARCHK(opf_vec_axpby(c, 1.0 / eps, xe, 1.0 / eps, vec(j + 1)));
        ARCHK(opf_vec_axpby(c, -1.0 / eps, P0, 1.0, vec(j + 1)));
        rep->products += 1;
        for (int i = 0; i <= j; ++i) {
            ARCHK(opf_vec_dot(c, vec(j + 1), vec(i), &H[(size_t)i * m + j]));
            ARCHK(opf_vec_axpby(c, -H[(size_t)i * m + j], vec(i), 1.0, vec(j + 1)));
        }
        double hn = 0.0;
        ARCHK(nrm(vec(j + 1), &hn));
        H[(size_t)(j + 1) * m + j] = hn;
        const int k = j + 1;
        if (k % check_every == 0 || k == m || hn == 0.0) {
            std::vector<double> hk((size_t)k * k), er(k), ei(k);
            for (int i = 0; i < k; ++i)
                for (int q = 0; q < k; ++q) hk[(size_t)i * k + q] = H[(size_t)i * m + q];
            ARCHK(opf_hessenberg_eigvals(hk.data(), k, er.data(), ei.data()));
            const int ne = std::min(nev, k);
            for (int i = 0; i < nev; ++i) {
                ritz_re[i] = i < ne ? er[i] : 0.0;
                ritz_im[i] = i < ne ? ei[i] : 0.0;
            }
            rep->checks += 1;
            bool done = hn == 0.0;
            if (have_prev && (int)prev.size() == 2 * ne) {
                double dmax = 0.0;
                for (int i = 0; i < ne; ++i) dmax = std::max(dmax, std::hypot(er[i] - prev[2 * i], ei[i] - prev[2 * i + 1]));
                if (dmax <= tol * std::hypot(er[0], ei[0])) done = true;
            }
            prev.assign(2 * ne, 0.0);
            for (int i = 0; i < ne; ++i) {
                prev[2 * i] = er[i];
                prev[2 * i + 1] = ei[i];
            }
            have_prev = true;
            if (done) {
                rep->converged = 1;
                break;
            }
        }
        if (hn == 0.0) break;
        ARCHK(opf_vec_axpby(c, 1.0 / hn, vec(j + 1), 0.0, vec(j + 1)));
    }
#undef ARCHK
    if (hess) std::copy(H.begin(), H.end(), hess);
    return OPF_OK;
}

opf_status opf_nk_workspace_size(const opf_ctx* c, int32_t m, int32_t preconditioned, size_t* bytes) {
    if (!c || !bytes || m < 1) return OPF_E_INVALID;
    *bytes = (size_t)(m + 6 + (preconditioned ? m : 0)) * 3 * field_entries(c) * 16;
    return OPF_OK;
}

// Newton-Krylov travelling-wave search.  Vectors of the (possibly extended)
// system are a device field plus a host scalar, the speed part (zero when
// the speed is fixed); their inner product is the energy inner product plus
// the product of the speed parts.
opf_status opf_nk_solve(opf_ctx* c, void* x_dev, double T, double* cw_io, const opf_nk_opts* o,
                        void* krylov_dev, size_t krylov_bytes, opf_nk_report* rep) {
    if (!c || !x_dev || !cw_io || !o || !krylov_dev || !rep) return OPF_E_INVALID;
    if (!std::isfinite(*cw_io) || o->max_jvps < 1 || o->gmres_m < 1) return OPF_E_INVALID;
    const int m = o->gmres_m;
    const bool pre = o->precond != nullptr;
    size_t need = 0;
    if (opf_nk_workspace_size(c, m, pre ? 1 : 0, &need) != OPF_OK || krylov_bytes < need) return OPF_E_NOMEM;
    if (o->record_capacity < 0 || (o->record_capacity > 0 && !o->record_dev)) return OPF_E_INVALID;
    *rep = opf_nk_report{};
    const bool hook = o->hookstep != 0;
    if (hook && pre) {
        c->err = "the hookstep is not combined with a preconditioner";
        return OPF_E_UNSUPPORTED;
    }
    const bool free_c = o->free_speed != 0;
    const double freeze = o->speed_freeze > 0 ? o->speed_freeze : 1e-6;
    const bool fallback = pre && !o->no_fallback;
    const int max_hook = o->max_hook > 0 ? o->max_hook : 12;
    const double delta_max = o->tr_delta_max > 0 ? o->tr_delta_max : INFINITY;
    double delta = o->tr_delta0;
    const size_t total = 3 * field_entries(c);
    const size_t vb = total * 16;  // bytes per field
    unsigned char* base = static_cast<unsigned char*>(krylov_dev);
    auto vec = [&](int i) { return static_cast<void*>(base + (size_t)i * vb); };
    // flexible GMRES keeps the preconditioned directions z_j = P(v_j)
    auto zvec = [&](int j) { return static_cast<void*>(base + (size_t)(m + 6 + j) * vb); };
    unsigned char* rec = static_cast<unsigned char*>(o->record_dev);
    void* F0 = vec(m + 1);   // F(x, c_w)
    void* tmp = vec(m + 2);  // x + eps v, then F(x + eps v)
    void* w = vec(m + 3);    // Arnoldi vector / J v
    void* dx = vec(m + 4);   // Newton update
    void* dzx = vec(m + 5);  // d_z x, the phase-condition vector
    std::vector<double> sv(m + 1, 0.0), sz(m, 0.0);  // speed parts of v_j, z_j
    double sw = 0.0, sdx = 0.0;
    double* x = static_cast<double*>(x_dev);
    double cw = *cw_io;
    auto dot = [&](const void* a, double sa, const void* b, double sb, double* out) {
        const opf_status st = opf_vec_dot(c, a, b, out);
        *out += sa * sb;
        return st;
    };
    auto nrm = [&](const void* a, double sa, double* out) {
        double s2 = 0.0;
        const opf_status st = dot(a, sa, a, sa, &s2);
        *out = std::sqrt(std::max(s2, 0.0));
        return st;
    };
#define NKCHK(call)                      \
    do {                                 \
        const opf_status st_ = (call);   \
        if (st_ != OPF_OK) return st_;   \
    } while (0)
    double fn = 0.0, xn = 0.0;
    NKCHK(opf_newton_residual(c, x, T, cw * T, F0, &fn));
    rep->residual_evals = 1;
    NKCHK(opf_vec_dot(c, x, x, &xn));
    xn = std::sqrt(std::max(xn, 0.0));
    rep->residual_history[0] = fn / xn;
    rep->residual = fn / xn;
    int it = 0;
    for (; it < o->max_newton && rep->residual > o->tol; ++it) {
        const int jv0 = rep->jvps;  // products at the start of this Newton step
        // the speed is solved for only where x has axial structure
        bool active = false;
        if (free_c) {
            hipLaunchKernelGGL(k_ddz, dim3((total + 255) / 256), dim3(256), 0, c->stream, x,
                               static_cast<double*>(dzx), c->p.N, c->nk, c->p.K, total, c->p.alpha);
            HIPCHK(c, hipGetLastError());
            double dn = 0.0;
            NKCHK(nrm(dzx, 0.0, &dn));
            active = dn > freeze * xn;
            if (!active) rep->frozen_steps += 1;
        }
        const double Xn = free_c ? std::sqrt(xn * xn + cw * cw) : xn;
        // J (v, s) = (F(x + eps v, c_w + eps s) - F(x, c_w)) / eps, plus the
        // phase row <d_z x, v> as its speed part; into (w, sw)
        auto jv = [&](const void* v, double& s, double vnorm) -> opf_status {
            if (!active) s = 0.0;
            const double eps = o->fd_eps * std::max(Xn, 1.0) / vnorm;
            NKCHK(opf_vec_axpby(c, 1.0, x, 0.0, tmp));
            NKCHK(opf_vec_axpby(c, eps, v, 1.0, tmp));
            HIPCHK(c, hipMemcpyAsync(w, tmp, vb, hipMemcpyDeviceToDevice, c->stream));
            NKCHK(opf_newton_residual(c, w, T, (cw + eps * s) * T, tmp, nullptr));
            NKCHK(opf_vec_axpby(c, -1.0 / eps, F0, 1.0 / eps, tmp));
            HIPCHK(c, hipMemcpyAsync(w, tmp, vb, hipMemcpyDeviceToDevice, c->stream));
            sw = 0.0;
            if (active) NKCHK(opf_vec_dot(c, dzx, v, &sw));
            rep->jvps += 1;
            // (z, J_x z) training pairs: products that move the state only
            if (rec && s == 0.0 && rep->recorded < o->record_capacity) {
                unsigned char* slot = rec + (size_t)rep->recorded * 2 * vb;
                HIPCHK(c, hipMemcpyAsync(slot, v, vb, hipMemcpyDeviceToDevice, c->stream));
                HIPCHK(c, hipMemcpyAsync(slot + vb, w, vb, hipMemcpyDeviceToDevice, c->stream));
                rep->recorded += 1;
            }
            return OPF_OK;
        };
        // (w, sw) = a (v, s) + b (w, sw)
        auto axpby_w = [&](double a, const void* v, double s) -> opf_status {
            NKCHK(opf_vec_axpby(c, a, v, 1.0, w));
            sw += a * s;
            return OPF_OK;
        };
        if (hook) {
            // one Arnoldi cycle from v_1 = -F / ||F||; Hr keeps the raw
            // Hessenberg matrix, Hw its Givens-rotated copy for the estimate
            NKCHK(opf_vec_axpby(c, -1.0 / fn, F0, 0.0, vec(0)));
            sv[0] = 0.0;
            std::vector<double> Hr((size_t)(m + 1) * m, 0.0), Hw((size_t)(m + 1) * m, 0.0);
            std::vector<double> cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
            g[0] = fn;
            int k = 0;
            for (int j = 0; j < m; ++j) {
                NKCHK(jv(vec(j), sv[j], 1.0));
                for (int i = 0; i <= j; ++i) {
                    NKCHK(dot(w, sw, vec(i), sv[i], &Hr[(size_t)i * m + j]));
                    NKCHK(axpby_w(-Hr[(size_t)i * m + j], vec(i), sv[i]));
                }
                double hn = 0.0;
                NKCHK(nrm(w, sw, &hn));
                Hr[(size_t)(j + 1) * m + j] = hn;
                for (int i = 0; i <= j + 1; ++i) Hw[(size_t)i * m + j] = Hr[(size_t)i * m + j];
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * Hw[(size_t)i * m + j] + sn[i] * Hw[(size_t)(i + 1) * m + j];
                    Hw[(size_t)(i + 1) * m + j] = -sn[i] * Hw[(size_t)i * m + j] + cs[i] * Hw[(size_t)(i + 1) * m + j];
                    Hw[(size_t)i * m + j] = t;
                }
                const double d = std::hypot(Hw[(size_t)j * m + j], hn);
                cs[j] = d == 0.0 ? 1.0 : Hw[(size_t)j * m + j] / d;
                sn[j] = d == 0.0 ? 0.0 : hn / d;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                k = j + 1;
                rep->gmres_iterations += 1;
                if (std::fabs(g[k]) <= o->gmres_tol * fn || hn == 0.0 || rep->jvps - jv0 >= o->max_jvps) break;
                NKCHK(opf_vec_axpby(c, 1.0 / hn, w, 0.0, vec(j + 1)));
                sv[j + 1] = sw / hn;
            }
            std::vector<double> hb((size_t)(k + 1) * k), y(k);
            for (int i = 0; i <= k; ++i)
                for (int j = 0; j < k; ++j) hb[(size_t)i * k + j] = Hr[(size_t)i * m + j];
            double mu = 0.0, r = 0.0;
            if (!(delta > 0)) {
                NKCHK(opf_hookstep_solve(hb.data(), k, fn, INFINITY, y.data(), &mu, &r));
                double l2 = 0.0;
                for (double v : y) l2 += v * v;
                delta = std::sqrt(l2);
            }
            bool accepted = false;
            double fnew = 0.0, cnew = cw;
            for (int trial = 0; trial < max_hook; ++trial) {
                NKCHK(opf_hookstep_solve(hb.data(), k, fn, delta, y.data(), &mu, &r));
                double dn2 = 0.0;
                for (double v : y) dn2 += v * v;
                const double dn = std::sqrt(dn2);
                NKCHK(opf_vec_axpby(c, 1.0, x, 0.0, w));
                cnew = cw;
                for (int i = 0; i < k; ++i) {
                    NKCHK(opf_vec_axpby(c, y[i], vec(i), 1.0, w));
                    cnew += y[i] * sv[i];
                }
                NKCHK(trial_residual(c, w, T, cnew * T, tmp, &fnew));
                rep->residual_evals += 1;
                rep->hook_trials += 1;
                const double den = fn * fn - r * r;
                const double rho = den > 0 ? (fn * fn - fnew * fnew) / den : -INFINITY;
                if (rho >= 0.1) {
                    accepted = true;
                    if (rho > 0.75 && dn >= 0.99 * delta) delta = std::min(2.0 * delta, delta_max);
                    else if (rho < 0.25) delta = 0.5 * dn;
                    break;
                }
                delta = 0.5 * dn;
            }
            rep->tr_delta = delta;
            if (!accepted) {
                rep->stalled = 1;
                break;
            }
            NKCHK(opf_vec_axpby(c, 1.0, w, 0.0, x));
            cw = cnew;
            HIPCHK(c, hipMemcpyAsync(F0, tmp, vb, hipMemcpyDeviceToDevice, c->stream));
            fn = fnew;
            NKCHK(opf_vec_dot(c, x, x, &xn));
            xn = std::sqrt(std::max(xn, 0.0));
            rep->residual = fn / xn;
            if (it + 1 < 32) rep->residual_history[it + 1] = rep->residual;
            continue;
        }
        // GMRES(m) for J (dx, sdx) = (-F0, 0) from zero, restarted; with the
        // preconditioner, one flexible cycle of at most m products.  Returns
        // whether the relative tolerance was reached.
        auto gmres = [&](bool use_pre, bool& reached) -> opf_status {
            NKCHK(opf_vec_axpby(c, 0.0, F0, 0.0, dx));
            sdx = 0.0;
            reached = false;
            const double bn = fn;
            const int start = rep->jvps;
            const int left = o->max_jvps - (start - jv0);  // this Newton step's remaining products
            const int cap = use_pre ? std::min(left, m) : left;
            int restarts = 0;
            while (true) {
                // r = -F0 - J dx
                double beta = 0.0;
                sv[0] = 0.0;
                if (restarts == 0) {
                    NKCHK(opf_vec_axpby(c, -1.0, F0, 0.0, vec(0)));
                } else {
                    double dxn = 0.0;
                    NKCHK(nrm(dx, sdx, &dxn));
                    NKCHK(jv(dx, sdx, dxn));
                    NKCHK(opf_vec_axpby(c, -1.0, F0, 0.0, vec(0)));
                    NKCHK(opf_vec_axpby(c, -1.0, w, 1.0, vec(0)));
                    sv[0] = -sw;
                }
                NKCHK(nrm(vec(0), sv[0], &beta));
                if (beta <= o->gmres_tol * bn) {
                    reached = true;
                    break;
                }
                if (rep->jvps - start >= cap) break;
                NKCHK(opf_vec_axpby(c, 0.0, vec(0), 1.0 / beta, vec(0)));
                sv[0] /= beta;
                std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
                auto Hh = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
                g[0] = beta;
                int k = 0;
                for (int j = 0; j < m; ++j) {
                    if (use_pre) {
                        double zn = 0.0;
                        NKCHK(opf_precondition(c, o->precond, vec(j), zvec(j)));
                        sz[j] = sv[j];  // the speed part passes unchanged
                        rep->precond_applies += 1;
                        NKCHK(nrm(zvec(j), sz[j], &zn));
                        if (!(zn > 0.0) || !std::isfinite(zn)) return OPF_E_NUMERIC;
                        NKCHK(jv(zvec(j), sz[j], zn));
                    } else {
                        NKCHK(jv(vec(j), sv[j], 1.0));
                    }
                    for (int i = 0; i <= j; ++i) {
                        NKCHK(dot(w, sw, vec(i), sv[i], &Hh(i, j)));
                        NKCHK(axpby_w(-Hh(i, j), vec(i), sv[i]));
                    }
                    double hn = 0.0;
                    NKCHK(nrm(w, sw, &hn));
                    Hh(j + 1, j) = hn;
                    for (int i = 0; i < j; ++i) {
                        const double t = cs[i] * Hh(i, j) + sn[i] * Hh(i + 1, j);
                        Hh(i + 1, j) = -sn[i] * Hh(i, j) + cs[i] * Hh(i + 1, j);
                        Hh(i, j) = t;
                    }
                    const double d = std::hypot(Hh(j, j), Hh(j + 1, j));
                    cs[j] = d == 0.0 ? 1.0 : Hh(j, j) / d;
                    sn[j] = d == 0.0 ? 0.0 : Hh(j + 1, j) / d;
                    Hh(j, j) = d;
                    Hh(j + 1, j) = 0.0;
                    g[j + 1] = -sn[j] * g[j];
                    g[j] = cs[j] * g[j];
                    k = j + 1;
                    rep->gmres_iterations += 1;
                    if (std::fabs(g[k]) <= o->gmres_tol * bn || hn == 0.0 || rep->jvps - start >= cap) break;
                    NKCHK(opf_vec_axpby(c, 1.0 / hn, w, 0.0, vec(j + 1)));
                    sv[j + 1] = sw / hn;
                }
                std::vector<double> y(k, 0.0);
                for (int i = k - 1; i >= 0; --i) {
                    double acc = g[i];
                    for (int j2 = i + 1; j2 < k; ++j2) acc -= Hh(i, j2) * y[j2];
                    y[i] = acc / Hh(i, i);
                }
                for (int i = 0; i < k; ++i) {
                    NKCHK(opf_vec_axpby(c, y[i], use_pre ? zvec(i) : vec(i), 1.0, dx));
                    sdx += y[i] * (use_pre ? sz[i] : sv[i]);
                }
                ++restarts;
                if (std::fabs(g[k]) <= o->gmres_tol * bn) {
                    reached = true;
                    break;
                }
                if (rep->jvps - start >= cap || use_pre) break;
            }
            return OPF_OK;
        };
        // backtracking line search on ||F|| along (dx, sdx); the candidate
        // stays in (w, tmp); returns whether ||F|| decreased
        double fnew = 0.0, cnew = cw;
        auto line_search = [&](bool& lowered) -> opf_status {
            double lam = 1.0;
            while (true) {
                NKCHK(opf_vec_axpby(c, 1.0, x, 0.0, w));
                NKCHK(opf_vec_axpby(c, lam, dx, 1.0, w));
                cnew = cw + lam * sdx;
                NKCHK(trial_residual(c, w, T, cnew * T, tmp, &fnew));
                rep->residual_evals += 1;
                if (fnew < fn || lam < 1e-3) break;
                lam *= 0.5;
            }
            if (!std::isfinite(fnew)) return OPF_E_NUMERIC;  // even the shortest step left the stable range
            lowered = fnew < fn;
            return OPF_OK;
        };
        bool reached = false, lowered = false;
        NKCHK(gmres(pre, reached));
        if (pre && fallback && !reached) {  // the network's directions did not solve the step
            rep->fallbacks += 1;
            NKCHK(gmres(false, reached));
            NKCHK(line_search(lowered));
        } else {
            NKCHK(line_search(lowered));
            if (pre && fallback && !lowered) {  // nor lowered ||F||: redo the step without it
                rep->fallbacks += 1;
                NKCHK(gmres(false, reached));
                NKCHK(line_search(lowered));
            }
        }
        NKCHK(opf_vec_axpby(c, 1.0, w, 0.0, x));
        cw = cnew;
        HIPCHK(c, hipMemcpyAsync(F0, tmp, vb, hipMemcpyDeviceToDevice, c->stream));
        fn = fnew;
        NKCHK(opf_vec_dot(c, x, x, &xn));
        xn = std::sqrt(std::max(xn, 0.0));
        rep->residual = fn / xn;
        if (it + 1 < 32) rep->residual_history[it + 1] = rep->residual;
    }
#undef NKCHK
    rep->newton_iterations = it;
    rep->converged = rep->residual <= o->tol ? 1 : 0;
    rep->speed = cw;
    *cw_io = cw;
    return OPF_OK;
}

}  // extern "C"

namespace {
// Probe i of a seed: unit normals, spectrum of a real field, unit energy norm.
opf_status make_probe(opf_ctx* c, double* z, int i, uint64_t seed) {
    const size_t total = 3 * field_entries(c);
    hipLaunchKernelGGL(k_noise, dim3((total + 255) / 256), dim3(256), 0, c->stream, z, total,
                       seed * 0x2545F4914F6CDD1Dull + (uint64_t)i * 0xD1B54A32D192ED03ull);
    hipLaunchKernelGGL(k_realfield, dim3((3 * c->p.K * c->p.N + 255) / 256), dim3(256), 0, c->stream, z, c->p.N,
                       c->p.M, c->nk, c->p.K);
    HIPCHK(c, hipGetLastError());
    double zn2 = 0.0;
    opf_status st = opf_vec_dot(c, z, z, &zn2);
    if (st != OPF_OK) return st;
    if (!(zn2 > 0.0)) return OPF_E_NUMERIC;
    return opf_vec_axpby(c, 0.0, z, 1.0 / std::sqrt(zn2), z);
}
}  // namespace

extern "C" {

}  // extern "C"

// Work vectors of opf_probe_pairs_noalloc: a file-scope device array.  In
// host code `scratch` only names the symbol; its device address on the
// current device comes from hipGetSymbolAddress, taken once per device on
// the first call there and kept (each device holds its own copy of the
// array until the process ends).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
// F = shift(Phi_T(x), -shift) - x with the steps launched one kernel at a
// time (the same kernels and arguments as the step graph, which is neither
// captured nor instantiated here).
opf_status residual_eager(opf_ctx* c, const void* x, double T, double shift, void* F) {
    if (!(T >= 0)) return OPF_E_INVALID;
    const int nsteps = (int)std::lround(T / c->p.dt);
    opf_status st = opf_set_state(c, x);
    if (st != OPF_OK) return st;
    for (int i = 0; i < nsteps; ++i)
        if ((st = enqueue_step(c, c->stream)) != OPF_OK) return st;
    if (nsteps > 0) c->pc_valid = true;
    const size_t total = 3 * field_entries(c);
    hipLaunchKernelGGL(k_shift_sub, dim3((total + 255) / 256), dim3(256), 0, c->stream, c->u,
                       static_cast<const double*>(x), static_cast<double*>(F), c->p.N, c->nk, c->p.K, total,
                       c->p.alpha, shift);
    HIPCHK(c, hipGetLastError());
    return OPF_OK;
}

// The probes of opf_probe_pairs with three work vectors at work_dev; eager
// selects the residual without the step graph.
opf_status probe_pairs_impl(opf_ctx* c, const void* x_dev, double T, double shift, int32_t n, uint64_t seed,
                            double fd_eps, void* pairs_dev, void* work_dev, bool eager) {
    const size_t total = 3 * field_entries(c);
    const size_t vb = total * 16;
    unsigned char* w = static_cast<unsigned char*>(work_dev);
    void* F0 = w;
    void* tmp = w + vb;
    void* F1 = w + 2 * vb;
    auto resid = [&](const void* x, void* F) {
        return eager ? residual_eager(c, x, T, shift, F) : opf_newton_residual(c, x, T, shift, F, nullptr);
    };
    opf_status st = resid(x_dev, F0);
    if (st != OPF_OK) return st;
    double xn2 = 0.0;
    if ((st = opf_vec_dot(c, x_dev, x_dev, &xn2)) != OPF_OK) return st;
    const double eps = fd_eps * std::max(std::sqrt(xn2), 1.0);
    unsigned char* out = static_cast<unsigned char*>(pairs_dev);
    for (int i = 0; i < n; ++i) {
        double* z = reinterpret_cast<double*>(out + (size_t)i * 2 * vb);
        void* jz = out + (size_t)i * 2 * vb + vb;
        if ((st = make_probe(c, z, i, seed)) != OPF_OK) return st;
        if ((st = opf_vec_axpby(c, 1.0, x_dev, 0.0, tmp)) != OPF_OK) return st;
        if ((st = opf_vec_axpby(c, eps, z, 1.0, tmp)) != OPF_OK) return st;
        if ((st = resid(tmp, F1)) != OPF_OK) return st;
        HIPCHK(c, hipMemcpyAsync(jz, F1, vb, hipMemcpyDeviceToDevice, c->stream));
        if ((st = opf_vec_axpby(c, -1.0 / eps, F0, 1.0 / eps, jz)) != OPF_OK) return st;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return OPF_OK;
}

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[NOALLOC_MAX_DEVICES] = {};

opf_status scratch_on_current_device(opf_ctx* c, void** out) {
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        c->err = "no-allocation scratch: device index out of range";
        return OPF_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (he != hipSuccess || !p) {
            c->err = std::string("no-allocation scratch: hipGetSymbolAddress: ") + hipGetErrorString(he);
            return OPF_E_HIP;
        }
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return OPF_OK;
}
}  // namespace

extern "C" {

opf_status opf_probe_pairs(opf_ctx* c, const void* x_dev, double T, double shift, int32_t n, uint64_t seed,
                           double fd_eps, void* pairs_dev, void* work_dev) {
    if (!c || !x_dev || !pairs_dev || !work_dev || n < 1 || !(fd_eps > 0.0)) return OPF_E_INVALID;
    return probe_pairs_impl(c, x_dev, T, shift, n, seed, fd_eps, pairs_dev, work_dev, false);
}

opf_status opf_probe_pairs_noalloc(opf_ctx* c, const void* x_dev, double T, double shift, int32_t n,
                                   uint64_t seed, double fd_eps, void* pairs_dev) {
    if (!c || !x_dev || !pairs_dev || n < 1 || !(fd_eps > 0.0)) return OPF_E_INVALID;
    const size_t need = 3 * (3 * field_entries(c) * 16);
    if (need > NOALLOC_SCRATCH_BYTES) {
        c->err = "opf_probe_pairs_noalloc: three fields of this grid take " + std::to_string(need) +
                 " bytes, more than the " + std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte scratch";
        return OPF_E_INVALID;
    }
    void* w = nullptr;
    const opf_status st = scratch_on_current_device(c, &w);
    if (st != OPF_OK) return st;
    return probe_pairs_impl(c, x_dev, T, shift, n, seed, fd_eps, pairs_dev, w, true);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Ensembles: members of equal (N, M, K, mp, precision) form a class; each
// kernel of the step runs once per class over all its members (grid.y =
// member, argument records in device memory), and the whole step of every
// class is one captured graph.
struct EnsClass {
    int N = 0, M = 0, K = 0, mp = 0, precision = 0, gm = 1;
    int tz = DEFAULT_TZ, ztile = DEFAULT_ZTILE;  // transform tile shapes
    std::vector<int> idx;                   // member indices
    NLArgs* nl[2] = {nullptr, nullptr};     // device argument records, NL(u^n), NL(u^p)
    SolveArgs* sv[2] = {nullptr, nullptr};  // predictor, corrector
    double tuned_us = 0.0;                  // per-step time of the class at its tile choice
};

struct opf_ensemble {
    std::vector<opf_ctx*> members;
    std::vector<EnsClass> classes;
    hipStream_t stream = nullptr, cap = nullptr;
    hipGraphExec_t graph = nullptr;
    std::string err;
};

namespace {

size_t ens_args_bytes(int count) {
    return (size_t)count * (2 * sizeof(NLArgs) + 2 * sizeof(SolveArgs) + 2 * 64);
}

size_t ens_layout(const opf_params* mem, int count, std::vector<size_t>* offs, std::vector<size_t>* sizes) {
    size_t o = 0;
    for (int i = 0; i < count; ++i) {
        size_t b = 0;
        if (opf_workspace_size(&mem[i], &b) != OPF_OK) return 0;
        if (offs) offs->push_back(o);
        if (sizes) sizes->push_back(b);
        o = align_up(o + b);
    }
    // argument records: 2 NL + 2 solve records per member, each class's two
    // groups padded to 64 bytes (at most count classes)
    o = align_up(o + ens_args_bytes(count));
    return o;
}

// Upload the argument records of class k with the current tile choice.
opf_status ens_upload(opf_ensemble* e, EnsClass& k, hipStream_t s) {
    std::vector<NLArgs> nl0, nl1;
    std::vector<SolveArgs> sp, sc;
    for (int i : k.idx) {
        opf_ctx* c = e->members[i];
        c->gm = k.gm;
        c->tz = k.tz;
        c->ztile = k.ztile;
        const bool mixed = c->p.precision == OPF_MIXED;
        const void* uin = mixed ? (const void*)c->u32 : (const void*)c->u;
        const void* upin = mixed ? (const void*)c->up32 : (const void*)c->up;
        nl0.push_back(nl_args(c, uin, c->w, c->Nn));
        nl1.push_back(nl_args(c, upin, c->w, c->Np));
        SolveArgs a = solve_args(c, OPF_SOLVE_PRED);
        a.u0 = c->u;
        a.n0 = c->Nn;
        a.u_out = mixed ? nullptr : c->up;
        a.u_out32 = mixed ? c->up32 : nullptr;
        a.w_out = c->w;
        sp.push_back(a);
        SolveArgs b = solve_args(c, OPF_SOLVE_CORR);
        b.u0 = c->u;
        b.n0 = c->Nn;
        b.n1 = c->Np;
        b.u_out = c->u;
        b.u_out32 = mixed ? c->u32 : nullptr;
        b.w_out = c->w;
        sc.push_back(b);
    }
    const size_t n = k.idx.size();
    hipError_t he = hipMemcpyAsync(k.nl[0], nl0.data(), n * sizeof(NLArgs), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipMemcpyAsync(k.nl[1], nl1.data(), n * sizeof(NLArgs), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipMemcpyAsync(k.sv[0], sp.data(), n * sizeof(SolveArgs), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipMemcpyAsync(k.sv[1], sc.data(), n * sizeof(SolveArgs), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);  // host vectors go out of scope
    if (he != hipSuccess) {
        e->err = std::string("ensemble upload: ") + hipGetErrorString(he);
        return OPF_E_HIP;
    }
    return OPF_OK;
}

// ---- tile cache (JSON) --------------------------------------------------
// {"version": 1, "classes": [{"N": .., "M": .., "K": .., "mp": .., "precision": ..,
//   "members": .., "gm": .., "tz": .., "ztile": .., "us_per_step": ..,
//   "candidates": [{"gm": .., "tz": .., "ztile": .., "us_per_step": ..}, ...]}, ...]}
// A minimal reader: objects, arrays, numbers, strings and literals.
struct JVal {
    enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal* get(const char* key) const {
        for (const auto& kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const char* p;
    const char* end;
    bool ok = true;
    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')) ++p;
    }
    bool lit(const char* w) {
        const size_t n = std::strlen(w);
        if ((size_t)(end - p) >= n && std::strncmp(p, w, n) == 0) {
            p += n;
            return true;
        }
        return false;
    }
    JVal value(int depth) {
        JVal v;
        ws();
        if (!ok || p >= end || depth > 32) {
            ok = false;
            return v;
        }
        if (*p == '{') {
            v.kind = JVal::OBJ;
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
                return v;
            }
            while (ok) {
                ws();
                JVal k = value(depth + 1);
                if (k.kind != JVal::STR) { ok = false; break; }
                ws();
                if (p >= end || *p != ':') { ok = false; break; }
                ++p;
                v.obj.emplace_back(k.str, value(depth + 1));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == '}') { ++p; break; }
                ok = false;
            }
        } else if (*p == '[') {
            v.kind = JVal::ARR;
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
                return v;
            }
            while (ok) {
                v.arr.push_back(value(depth + 1));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == ']') { ++p; break; }
                ok = false;
            }
        } else if (*p == '"') {
            v.kind = JVal::STR;
            ++p;
            while (p < end && *p != '"') {
                if (*p == '\\' && p + 1 < end) ++p;
                v.str += *p++;
            }
            if (p >= end) ok = false;
            else ++p;
        } else if (lit("true")) {
            v.kind = JVal::BOOL;
            v.num = 1.0;
        } else if (lit("false")) {
            v.kind = JVal::BOOL;
        } else if (lit("null")) {
        } else {
            char* q = nullptr;
            v.num = std::strtod(p, &q);
            if (q == p) ok = false;
            else {
                v.kind = JVal::NUM;
                p = q;
            }
        }
        return v;
    }
};

struct TileChoice {
    int N, M, K, mp, precision, gm, tz, ztile;
};

bool tiles_ok(const TileChoice& t) {
    return gm_ok(t.gm, t.mp) && t.gm <= t.M && tz_ok(t.tz, t.M) && ztile_ok(t.ztile, t.K);
}

// Parse a tile cache; false (with msg) on a malformed file or an
// inadmissible entry.
bool parse_tile_cache(const std::string& text, std::vector<TileChoice>& out, std::string& msg) {
    JParser ps{text.data(), text.data() + text.size()};
    const JVal root = ps.value(0);
    ps.ws();
    if (!ps.ok || ps.p != ps.end || root.kind != JVal::OBJ) {
        msg = "tile cache: not a JSON object";
        return false;
    }
    const JVal* cls = root.get("classes");
    if (!cls || cls->kind != JVal::ARR) {
        msg = "tile cache: no \"classes\" array";
        return false;
    }
    for (const JVal& c : cls->arr) {
        TileChoice t{};
        int* f[] = {&t.N, &t.M, &t.K, &t.mp, &t.precision, &t.gm, &t.tz, &t.ztile};
        const char* names[] = {"N", "M", "K", "mp", "precision", "gm", "tz", "ztile"};
        for (int i = 0; i < 8; ++i) {
            const JVal* v = c.kind == JVal::OBJ ? c.get(names[i]) : nullptr;
            // an integer in int range (casting a number outside it is undefined)
            if (!v || v->kind != JVal::NUM || !(std::fabs(v->num) < 1e9) || v->num != std::floor(v->num)) {
                msg = std::string("tile cache: class entry without integer \"") + names[i] + "\"";
                return false;
            }
            *f[i] = (int)v->num;
        }
        if (!tiles_ok(t)) {
            msg = "tile cache: inadmissible tiles for class N=" + std::to_string(t.N) + " M=" + std::to_string(t.M) +
                  " K=" + std::to_string(t.K);
            return false;
        }
        out.push_back(t);
    }
    return true;
}

std::string tile_cache_json(const std::vector<opf_tiles>& t, const std::vector<std::string>& candidates) {
    std::string js = "{\"version\": 1, \"classes\": [";
    for (size_t i = 0; i < t.size(); ++i) {
        char buf[320];
        std::snprintf(buf, sizeof buf,
                      "%s{\"N\": %d, \"M\": %d, \"K\": %d, \"mp\": %d, \"precision\": %d, \"members\": %d, "
                      "\"gm\": %d, \"tz\": %d, \"ztile\": %d, \"us_per_step\": %.3f",
                      i ? ", " : "", t[i].N, t[i].M, t[i].K, t[i].mp, t[i].precision, t[i].members, t[i].gm, t[i].tz,
                      t[i].ztile, t[i].us_per_step);
        js += buf;
        if (i < candidates.size()) js += ", \"candidates\": [" + candidates[i] + "]";
        js += "}";
    }
    return js + "]}";
}

bool read_file(const char* path, std::string& out) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return false;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) out.append(buf, n);
    std::fclose(f);
    return true;
}

bool write_file(const char* path, const std::string& text) {
    FILE* f = std::fopen(path, "wb");
    if (!f) return false;
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    return std::fclose(f) == 0 && ok;
}

// One predictor-corrector step of class k (all members, batched launches).
hipError_t ens_enqueue_class(opf_ensemble* e, const EnsClass& k, hipStream_t s) {
    opf_ctx* c0 = e->members[k.idx[0]];
    const int nm = (int)k.idx.size();
    NLArgs proto = nl_args(c0, c0->u, c0->w, c0->Nn);
    SolveArgs sproto = solve_args(c0, OPF_SOLVE_PRED);
    sproto.gm = k.gm;
    hipError_t he = hipSuccess;
    for (int half = 0; half < 2 && he == hipSuccess; ++half) {
        if (c0->p.nonlinear)
            for (int stage = 0; stage < 3 && he == hipSuccess; ++stage)
                he = launch_nonlinear_batch(proto, k.nl[half], nm, k.precision, stage, s);
        if (he == hipSuccess) he = launch_solve_batch(sproto, k.sv[half], nm, k.precision, s);
    }
    return he;
}

}  // namespace

extern "C" {

opf_status opf_ensemble_workspace_size(const opf_params* members, int32_t count, size_t* bytes) {
    if (!members || count < 1 || !bytes) return OPF_E_INVALID;
    for (int i = 0; i < count; ++i) {
        const opf_status st = validate(&members[i], nullptr);
        if (st != OPF_OK) return st;
    }
    *bytes = ens_layout(members, count, nullptr, nullptr);
    return *bytes ? OPF_OK : OPF_E_INVALID;
}

opf_status opf_ensemble_create(const opf_params* members, int32_t count, void* ws, size_t bytes,
                               void* hip_stream, const char* tune_cache_json, opf_ensemble** out) {
    if (!members || count < 1 || !ws || !out) return OPF_E_INVALID;
    *out = nullptr;
    std::vector<TileChoice> cached;
    if (tune_cache_json) {
        std::string text, msg;
        if (!read_file(tune_cache_json, text) || !parse_tile_cache(text, cached, msg)) return OPF_E_INVALID;
    }
    std::vector<size_t> offs, sizes;
    const size_t need = ens_layout(members, count, &offs, &sizes);
    if (!need) return OPF_E_INVALID;
    if (bytes < need) return OPF_E_NOMEM;
    if (reinterpret_cast<uintptr_t>(ws) % ALIGN != 0) return OPF_E_INVALID;
    opf_ensemble* e = new (std::nothrow) opf_ensemble();
    if (!e) return OPF_E_NOMEM;
    e->stream = static_cast<hipStream_t>(hip_stream);
    unsigned char* base = static_cast<unsigned char*>(ws);
    for (int i = 0; i < count; ++i) {
        opf_ctx* c = nullptr;
        const opf_status st = opf_create(&members[i], base + offs[i], sizes[i], hip_stream, &c);
        if (st != OPF_OK) {
            for (opf_ctx* m : e->members) opf_destroy(m);
            delete e;
            return st;
        }
        c->in_ensemble = true;
        e->members.push_back(c);
    }
    for (int i = 0; i < count; ++i) {
        const opf_params& p = e->members[i]->p;
        EnsClass* k = nullptr;
        for (EnsClass& q : e->classes)
            if (q.N == p.N && q.M == p.M && q.K == p.K && q.mp == p.mp && q.precision == p.precision &&
                e->members[q.idx[0]]->p.nonlinear == p.nonlinear)
                k = &q;
        if (!k) {
            e->classes.emplace_back();
            k = &e->classes.back();
            k->N = p.N;
            k->M = p.M;
            k->K = p.K;
            k->mp = p.mp;
            k->precision = p.precision;
            k->gm = default_gm(p.mp);
            k->ztile = default_ztile(p.precision);
            for (const TileChoice& t : cached)  // tiles from the cache, where it has the class
                if (t.N == p.N && t.M == p.M && t.K == p.K && t.mp == p.mp && t.precision == p.precision) {
                    k->gm = t.gm;
                    k->tz = t.tz;
                    k->ztile = t.ztile;
                }
        }
        k->idx.push_back(i);
    }
    unsigned char* args = base + ens_layout(members, count, nullptr, nullptr) - align_up(ens_args_bytes(count));
    size_t o = 0;
    for (EnsClass& k : e->classes) {
        const size_t n = k.idx.size();
        for (int h = 0; h < 2; ++h) {
            k.nl[h] = reinterpret_cast<NLArgs*>(args + o);
            o += n * sizeof(NLArgs);
        }
        o = (o + 63) / 64 * 64;
        for (int h = 0; h < 2; ++h) {
            k.sv[h] = reinterpret_cast<SolveArgs*>(args + o);
            o += n * sizeof(SolveArgs);
        }
        o = (o + 63) / 64 * 64;
        const opf_status st = ens_upload(e, k, e->stream);
        if (st != OPF_OK) {
            opf_ensemble_destroy(e);
            return st;
        }
    }
    *out = e;
    return OPF_OK;
}

opf_status opf_ensemble_destroy(opf_ensemble* e) {
    if (!e) return OPF_E_INVALID;
    if (e->graph) (void)hipGraphExecDestroy(e->graph);
    if (e->cap) (void)hipStreamDestroy(e->cap);
    for (opf_ctx* c : e->members) opf_destroy(c);
    delete e;
    return OPF_OK;
}

opf_status opf_ensemble_member(opf_ensemble* e, int32_t i, opf_ctx** out) {
    if (!e || !out || i < 0 || i >= (int)e->members.size()) return OPF_E_INVALID;
    *out = e->members[i];
    return OPF_OK;
}

opf_status opf_ensemble_step(opf_ensemble* e, int32_t nsteps) {
    if (!e || nsteps < 0) return OPF_E_INVALID;
    for (opf_ctx* c : e->members)
        if (!c->have_state) return OPF_E_STATE;
    if (!e->graph) {
        auto fail = [&](const char* what, hipError_t he) {
            e->err = std::string(what) + ": " + hipGetErrorString(he);
            return OPF_E_HIP;
        };
        hipError_t he = hipSuccess;
        if (!e->cap) he = hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking);
        if (he != hipSuccess) return fail("stream", he);
        hipGraph_t g = nullptr;
        he = hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal);
        if (he != hipSuccess) return fail("capture", he);
        hipError_t ke = hipSuccess;
        for (const EnsClass& k : e->classes)
            if (ke == hipSuccess) ke = ens_enqueue_class(e, k, e->cap);
        he = hipStreamEndCapture(e->cap, &g);
        if (ke != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail("launch", ke);
        }
        if (he != hipSuccess) return fail("capture", he);
        he = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (he != hipSuccess) {
            e->graph = nullptr;
            return fail("instantiate", he);
        }
    }
    for (int i = 0; i < nsteps; ++i) {
        const hipError_t he = hipGraphLaunch(e->graph, e->stream);
        if (he != hipSuccess) {
            e->err = std::string("graph launch: ") + hipGetErrorString(he);
            return OPF_E_HIP;
        }
    }
    return OPF_OK;
}

opf_status opf_probe_pairs_ensemble(opf_ensemble* e, const void* x_dev, double T, double shift, int32_t n,
                                    uint64_t seed, double fd_eps, void* pairs_dev, void* work_dev) {
    if (!e || e->members.empty() || !x_dev || !pairs_dev || !work_dev || n < 1 || !(fd_eps > 0.0))
        return OPF_E_INVALID;
    opf_ctx* c0 = e->members[0];
    for (opf_ctx* c : e->members) {
        const opf_params &a = c->p, &b = c0->p;
        if (a.N != b.N || a.M != b.M || a.K != b.K || a.mp != b.mp || a.alpha != b.alpha || a.Re != b.Re ||
            a.dt != b.dt || a.c != b.c || a.n_corr != b.n_corr || a.fixed_flux != b.fixed_flux ||
            a.precision != b.precision || a.nonlinear != b.nonlinear || c->r != c0->r)
            return OPF_E_INVALID;
    }
    if (!(T >= 0)) return OPF_E_INVALID;
    const size_t total = 3 * field_entries(c0);
    const size_t vb = total * 16;
    unsigned char* w = static_cast<unsigned char*>(work_dev);
    void* F0 = w;
    void* tmp = w + vb;
    void* F1 = w + 2 * vb;
    opf_status st = opf_newton_residual(c0, x_dev, T, shift, F0, nullptr);
    if (st != OPF_OK) return st;
    double xn2 = 0.0;
    if ((st = opf_vec_dot(c0, x_dev, x_dev, &xn2)) != OPF_OK) return st;
    const double eps = fd_eps * std::max(std::sqrt(xn2), 1.0);
    const int nsteps = (int)std::lround(T / c0->p.dt);
    const int B = (int)e->members.size();
    unsigned char* out = static_cast<unsigned char*>(pairs_dev);
    for (int i0 = 0; i0 < n; i0 += B) {
        const int nb = std::min(B, n - i0);
        for (int j = 0; j < B; ++j) {  // member j runs x + eps z_{i0+j} (idle members run x)
            if (j < nb) {
                double* z = reinterpret_cast<double*>(out + (size_t)(i0 + j) * 2 * vb);
                if ((st = make_probe(c0, z, i0 + j, seed)) != OPF_OK) return st;
                if ((st = opf_vec_axpby(c0, 1.0, x_dev, 0.0, tmp)) != OPF_OK) return st;
                if ((st = opf_vec_axpby(c0, eps, z, 1.0, tmp)) != OPF_OK) return st;
                if ((st = opf_set_state(e->members[j], tmp)) != OPF_OK) return st;
            } else if ((st = opf_set_state(e->members[j], x_dev)) != OPF_OK) {
                return st;
            }
        }
        if ((st = opf_ensemble_step(e, nsteps)) != OPF_OK) return st;
        for (int j = 0; j < nb; ++j) {  // J z = (shift(Phi_T(x + eps z), -s) - (x + eps z) - F(x)) / eps
            opf_ctx* c = e->members[j];
            const double* z = reinterpret_cast<const double*>(out + (size_t)(i0 + j) * 2 * vb);
            void* jz = out + (size_t)(i0 + j) * 2 * vb + vb;
            if ((st = opf_vec_axpby(c, 1.0, x_dev, 0.0, tmp)) != OPF_OK) return st;
            if ((st = opf_vec_axpby(c, eps, z, 1.0, tmp)) != OPF_OK) return st;
            hipLaunchKernelGGL(k_shift_sub, dim3((total + 255) / 256), dim3(256), 0, c->stream, c->u,
                               static_cast<const double*>(tmp), static_cast<double*>(F1), c->p.N, c->nk, c->p.K,
                               total, c->p.alpha, shift);
            HIPCHK(c, hipGetLastError());
            HIPCHK(c, hipMemcpyAsync(jz, F1, vb, hipMemcpyDeviceToDevice, c->stream));
            if ((st = opf_vec_axpby(c, -1.0 / eps, F0, 1.0 / eps, jz)) != OPF_OK) return st;
        }
    }
    if (hipStreamSynchronize(e->stream) != hipSuccess) return OPF_E_HIP;
    return OPF_OK;
}

opf_status opf_ensemble_tune(opf_ensemble* e, int32_t nsteps, char* report, size_t report_bytes) {
    if (!e || nsteps < 1) return OPF_E_INVALID;
    // members without a state run on laminar flow while the tiles are timed
    // (finite, representative data) and have no state afterwards
    std::vector<opf_ctx*> filled;
    for (opf_ctx* c : e->members)
        if (!c->have_state) {
            const size_t total = 3 * field_entries(c);
            hipLaunchKernelGGL(k_laminar, dim3((total + 255) / 256), dim3(256), 0, e->stream, c->u, c->u32,
                               c->t.r, c->p.N, c->nk, c->p.K, total);
            HIPCHK(c, hipGetLastError());
            opf_status st = refresh_derived(c);
            if (st != OPF_OK) return st;
            filled.push_back(c);
        }
    std::vector<opf_tiles> chosen;
    std::vector<std::string> cands;
    for (size_t ci = 0; ci < e->classes.size(); ++ci) {
        EnsClass& k = e->classes[ci];
        opf_ctx* c0 = e->members[k.idx[0]];
        std::string cand;
        // time one setting: nsteps batched steps of the class after a warm-up step
        auto time_it = [&](double* us) -> opf_status {
            opf_status st = ens_upload(e, k, e->stream);
            if (st != OPF_OK) return st;
            hipEvent_t a, b;
            HIPCHK(c0, hipEventCreate(&a));
            HIPCHK(c0, hipEventCreate(&b));
            hipError_t he = ens_enqueue_class(e, k, e->stream);
            if (he == hipSuccess) he = hipEventRecord(a, e->stream);
            for (int t = 0; t < nsteps && he == hipSuccess; ++t) he = ens_enqueue_class(e, k, e->stream);
            if (he == hipSuccess) he = hipEventRecord(b, e->stream);
            if (he == hipSuccess) he = hipEventSynchronize(b);
            float ms = 0.0f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, a, b);
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            if (he != hipSuccess) {
                e->err = std::string("tune: ") + hipGetErrorString(he);
                return OPF_E_HIP;
            }
            *us = 1e3 * ms / nsteps;
            char buf[128];
            std::snprintf(buf, sizeof buf, "%s{\"gm\": %d, \"tz\": %d, \"ztile\": %d, \"us_per_step\": %.3f}",
                          cand.empty() ? "" : ", ", k.gm, k.tz, k.ztile, *us);
            cand += buf;
            return OPF_OK;
        };
        // one tile dimension at a time, each from the best of the previous
        double best = 1e300;
        const int gms[] = {1, 2, 4}, tzs[] = {2, 4, 8}, zts[] = {4, 8, 16};
        for (int dim = 0; dim < 3; ++dim) {
            const int* vals = dim == 0 ? gms : dim == 1 ? tzs : zts;
            int* knob = dim == 0 ? &k.gm : dim == 1 ? &k.tz : &k.ztile;
            const int keep = *knob;
            int pick = keep;
            for (int i = 0; i < 3; ++i) {
                *knob = vals[i];
                const bool ok = dim == 0 ? gm_ok(k.gm, k.mp) && k.gm <= k.M
                              : dim == 1 ? tz_ok(k.tz, k.M) : ztile_ok(k.ztile, k.K);
                if (!ok) continue;
                double us = 0.0;
                const opf_status st = time_it(&us);
                if (st != OPF_OK) return st;
                if (us < best) {
                    best = us;
                    pick = vals[i];
                }
            }
            *knob = pick;
            (void)keep;
        }
        k.tuned_us = best;
        const opf_status st = ens_upload(e, k, e->stream);
        if (st != OPF_OK) return st;
        chosen.push_back(opf_tiles{k.N, k.M, k.K, k.mp, k.precision, (int)k.idx.size(), k.gm, k.tz, k.ztile, best});
        cands.push_back(cand);
    }
    for (opf_ctx* c : filled) c->have_state = false;
    if (e->graph) {  // recapture with the chosen tiles
        (void)hipGraphExecDestroy(e->graph);
        e->graph = nullptr;
    }
    const std::string js = tile_cache_json(chosen, cands);
    if (report && report_bytes) {
        std::strncpy(report, js.c_str(), report_bytes - 1);
        report[report_bytes - 1] = 0;
    }
    return OPF_OK;
}

opf_status opf_ensemble_tiles(const opf_ensemble* e, opf_tiles* out, int32_t capacity, int32_t* nclasses) {
    if (!e || !nclasses || capacity < 0 || (capacity > 0 && !out)) return OPF_E_INVALID;
    *nclasses = (int32_t)e->classes.size();
    for (int i = 0; i < std::min<int>(capacity, (int)e->classes.size()); ++i) {
        const EnsClass& k = e->classes[i];
        out[i] = opf_tiles{k.N, k.M, k.K, k.mp, k.precision, (int)k.idx.size(), k.gm, k.tz, k.ztile, k.tuned_us};
    }
    return OPF_OK;
}

opf_status opf_tile_cache_write(const opf_tiles* t, int32_t n, const char* path) {
    if (!t || n < 0 || !path) return OPF_E_INVALID;
    std::vector<opf_tiles> v(t, t + n);
    for (const opf_tiles& x : v)
        if (!tiles_ok(TileChoice{x.N, x.M, x.K, x.mp, x.precision, x.gm, x.tz, x.ztile})) return OPF_E_INVALID;
    return write_file(path, tile_cache_json(v, {})) ? OPF_OK : OPF_E_INVALID;
}

opf_status opf_tile_cache_read(const char* path, opf_tiles* out, int32_t capacity, int32_t* n) {
    if (!path || !n || capacity < 0 || (capacity > 0 && !out)) return OPF_E_INVALID;
    std::string text, msg;
    std::vector<TileChoice> v;
    if (!read_file(path, text) || !parse_tile_cache(text, v, msg)) return OPF_E_INVALID;
    *n = (int32_t)v.size();
    for (int i = 0; i < std::min<int>(capacity, (int)v.size()); ++i)
        out[i] = opf_tiles{v[i].N, v[i].M, v[i].K, v[i].mp, v[i].precision, 0, v[i].gm, v[i].tz, v[i].ztile, 0.0};
    return OPF_OK;
}

opf_status opf_autotune(const opf_params* cls, int32_t ncls, const char* cache_json_out) {
    if (!cls || ncls < 1 || !cache_json_out) return OPF_E_INVALID;
    constexpr int B = 8;  // members timed per class
    std::vector<opf_params> mem;
    for (int i = 0; i < ncls; ++i)
        for (int j = 0; j < B; ++j) mem.push_back(cls[i]);
    size_t bytes = 0;
    opf_status st = opf_ensemble_workspace_size(mem.data(), (int32_t)mem.size(), &bytes);
    if (st != OPF_OK) return st;
    void* ws = nullptr;
    hipStream_t s = nullptr;
    if (hipMalloc(&ws, bytes) != hipSuccess) return OPF_E_NOMEM;
    if (hipStreamCreate(&s) != hipSuccess) {
        (void)hipFree(ws);
        return OPF_E_HIP;
    }
    opf_ensemble* e = nullptr;
    st = opf_ensemble_create(mem.data(), (int32_t)mem.size(), ws, bytes, s, nullptr, &e);
    std::string js(1 << 16, '\0');
    if (st == OPF_OK) st = opf_ensemble_tune(e, 5, &js[0], js.size());
    if (e) opf_ensemble_destroy(e);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    (void)hipFree(ws);
    if (st != OPF_OK) return st;
    js.resize(std::strlen(js.c_str()));
    return write_file(cache_json_out, js) ? OPF_OK : OPF_E_INVALID;
}

const char* opf_ensemble_last_error(const opf_ensemble* e) { return e ? e->err.c_str() : "null ensemble"; }

}  // extern "C"
