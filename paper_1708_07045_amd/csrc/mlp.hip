// Learned importance-sampling proposal over ligand configurations: a 3-layer
// SiLU network on gfx950 with BF16 MFMA products and FP32 accumulation,
// trained by its own forward/backward kernels and Adam, plus the defensive
// mixture proposal and its inverse-CDF sampler.
//
// GEMMs use v_mfma_f32_16x16x16_bf16 through __builtin_amdgcn_mfma_f32_16x16x16bf16_1k.
// Operand layout per 64-lane wavefront (16 x 16 x 16 block):
//   A[i][k]: lane = i + 16*(k/4), element k%4      (row i, 4 consecutive k)
//   B[k][j]: lane = j + 16*(k/4), element k%4      (column j, 4 consecutive k)
//   D[i][j]: lane = j + 16*(i/4), element i%4
// so with both operands stored K-contiguous a lane loads 8 contiguous bytes.
// Every kernel is also instantiated with FP32 operands and activations
// (element type E = float; GEMMs on v_mfma_f32_16x16x4_f32, A[i][k] at lane
// i + 16 k and B[k][j] at lane j + 16 k of each 16 x 16 x 4 step, D as above):
// the same network in FP32 throughout, for checking gradients against an
// FP64 reference to FP32 rounding.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fftdg.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KP = 64;  // padded input width of the first layer

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// operand / activation element: BF16 bits (uint16_t) or FP32
template <typename E> __device__ __forceinline__ E to_e(float f);
template <> __device__ __forceinline__ uint16_t to_e<uint16_t>(float f) { return f2bf(f); }
template <> __device__ __forceinline__ float to_e<float>(float f) { return f; }
__device__ __forceinline__ float from_e(uint16_t h) { return bf2f(h); }
__device__ __forceinline__ float from_e(float f) { return f; }
__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// C[M][N] = A[M][K] * B[N][K]^T, E operands, FP32 accumulation.
// M, N multiples of 64; K multiple of 16; lda, ldb multiples of 4.
// mode 0: C (+ bias[n] if bias) -> Cout (fp32, ldc)
// mode 1: Z = C + bias[n] -> Cout; H = silu(Z) -> Hout (E, ldh)
template <typename E>
__global__ __launch_bounds__(256) void k_gemm(const E *__restrict__ A, int lda, const E *__restrict__ B, int ldb,
                                              int K, const float *__restrict__ bias, int mode,
                                              float *__restrict__ Cout, int ldc, E *__restrict__ Hout, int ldh) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32, n0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < K; k += 16) {
        if constexpr (sizeof(E) == 2) {
            bf16x4 fa[2], fb[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                fa[t] = *reinterpret_cast<const bf16x4 *>(A + (size_t)(m0 + t * 16 + r) * lda + k + kq);
                fb[t] = *reinterpret_cast<const bf16x4 *>(B + (size_t)(n0 + t * 16 + r) * ldb + k + kq);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
        } else {
            // four 16 x 16 x 4 steps; lane (r, q = lane / 16) supplies k + 4 s + q
            const int q = lane >> 4;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                float fa[2], fb[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    fa[t] = A[(size_t)(m0 + t * 16 + r) * lda + k + 4 * s4 + q];
                    fb[t] = B[(size_t)(n0 + t * 16 + r) * ldb + k + 4 * s4 + q];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = m0 + a * 16 + (lane >> 4) * 4 + e;
                const int j = n0 + b * 16 + (lane & 15);
                float v = acc[a][b][e];
                if (bias) v += bias[j];
                Cout[(size_t)i * ldc + j] = v;
                if (mode == 1) Hout[(size_t)i * ldh + j] = to_e<E>(silu(v));
            }
}

// rows idx[b] of X [N][n_in] (fp32) -> A0 [Bp][KP] (E), zero padded
template <typename E>
__global__ void k_gather(const float *__restrict__ X, int n_in, const int32_t *__restrict__ idx, int B, int Bp,
                         E *__restrict__ A0) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Bp * KP) return;
    const int b = e / KP, k = e - b * KP;
    float v = 0.f;
    if (b < B && k < n_in) v = X[(size_t)(idx ? idx[b] : b) * n_in + k];
    A0[e] = to_e<E>(v);
}

// y[b] = H3[b] . W4 + b4 (FP32 accumulation of E activations and
// weights), plus skip_scale times input column skip_col of the row (FP32)
// when skip_col >= 0
template <typename E>
__global__ void k_out(const E *__restrict__ H3, int W, const E *__restrict__ W4, const float *b4,
                      int B, const float *__restrict__ X, int n_in, const int32_t *__restrict__ idx, int skip_col,
                      float skip_scale, float *__restrict__ y) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float s = 0.f;
    for (int k = 0; k < W; ++k) s += from_e(H3[(size_t)b * W + k]) * from_e(W4[k]);
    const float sk = skip_col >= 0 ? skip_scale * X[(size_t)(idx ? idx[b] : b) * n_in + skip_col] : 0.f;
    y[b] = s + b4[0] + sk;
}

// dy = 2 w (y - t) / sum(w) and the loss; one workgroup, fixed reduction tree
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ y, const float *__restrict__ t_all,
                                              const float *__restrict__ w_all, const int32_t *__restrict__ idx, int B,
                                              float *__restrict__ dy, float *__restrict__ loss_out) {
    __shared__ float sw[256], sl[256];
    float a = 0.f, l = 0.f;
    for (int b = threadIdx.x; b < B; b += 256) {
        const int i = idx ? idx[b] : b;
        const float d = y[b] - t_all[i];
        a += w_all[i];
        l += w_all[i] * d * d;
    }
    sw[threadIdx.x] = a;
    sl[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sw[threadIdx.x] += sw[threadIdx.x + s];
            sl[threadIdx.x] += sl[threadIdx.x + s];
        }
        __syncthreads();
    }
    const float W = sw[0];
    for (int b = threadIdx.x; b < B; b += 256) {
        const int i = idx ? idx[b] : b;
        dy[b] = 2.f * w_all[i] * (y[b] - t_all[i]) / W;
    }
    if (threadIdx.x == 0) loss_out[0] = sl[0] / W;
}

// output layer gradients: dW4[k] = sum_b dy_b H3[b][k], db4 = sum_b dy_b
template <typename E>
__global__ void k_out_grad(const float *__restrict__ dy, const E *__restrict__ H3, int W, int B,
                           float *__restrict__ gW4, float *__restrict__ gb4) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > W) return;
    float s = 0.f;
    if (k < W)
        for (int b = 0; b < B; ++b) s += dy[b] * from_e(H3[(size_t)b * W + k]);
    else
        for (int b = 0; b < B; ++b) s += dy[b];
    if (k < W) gW4[k] = s; else gb4[0] = s;
}

// dZ[b][n] = dH[b][n] * silu'(Z[b][n]) with dH = dy_b W4[n] (from_out) or the
// given fp32 dH; writes E dZ [Bp][N] and its transpose [N][Bp] (rows
// b >= B are zero) and keeps fp32 dZ for the bias gradient.
template <typename E>
__global__ void k_dz(const float *__restrict__ dH, const float *__restrict__ dy, const E *__restrict__ W4,
                     const float *__restrict__ Z, int N, int B, int Bp, float *__restrict__ dZf, E *__restrict__ dZ,
                     E *__restrict__ dZt) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Bp * N) return;
    const int b = e / N, n = e - b * N;
    float v = 0.f;
    if (b < B) {
        const float g = dH ? dH[e] : dy[b] * from_e(W4[n]);
        v = g * dsilu(Z[e]);
    }
    dZf[e] = v;
    const E h = to_e<E>(v);
    dZ[e] = h;
    dZt[(size_t)n * Bp + b] = h;
}

// column sums: out[n] = sum_b M[b][n], b < B
__global__ void k_colsum(const float *__restrict__ M, int N, int B, float *__restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += M[(size_t)b * N + n];
    out[n] = s;
}

// transpose: out[c][r] = in[r][c], in [R][C]
template <typename E>
__global__ void k_transpose(const E *__restrict__ in, int R, int C, E *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= R * C) return;
    const int r = e / C, c = e - r * C;
    out[(size_t)c * R + r] = in[e];
}

// copy a [rows][cols_src] fp32 block into [rows][cols_dst] (first cols_src columns)
__global__ void k_copy_cols(const float *__restrict__ src, int rows, int cs, int cd, float *__restrict__ dst) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cd) return;
    const int r = e / cd, c = e - r * cd;
    dst[e] = src[(size_t)r * cs + c];
}

// Adam on the flat FP32 master parameters
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// E working copies of a weight matrix [R][C] into [R][ldd] (zero padded)
template <typename E>
__global__ void k_w_copy(const float *__restrict__ W, int R, int C, int ldd, E *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= R * ldd) return;
    const int r = e / ldd, c = e - r * ldd;
    out[e] = to_e<E>(c < C ? W[(size_t)r * C + c] : 0.f);
}

// Defensive mixture proposal over P configurations and inverse-CDF draws:
//   q_c = (1 - alpha) softmax(yhat / tau)_c + alpha / P       (FP64)
//   idx_k = smallest c with u_k * cdf[P-1] < cdf[c]
// One workgroup; the CDF is a fixed-order block scan.
__global__ __launch_bounds__(256) void k_proposal(const float *__restrict__ yhat, int P, double alpha, double tau,
                                                  int K, const double *__restrict__ u, int32_t *__restrict__ idx,
                                                  double *__restrict__ q, double *__restrict__ cdf) {
    __shared__ double sh[256];
    double mx = -INFINITY;
    for (int c = threadIdx.x; c < P; c += 256) mx = fmax(mx, (double)yhat[c] / tau);
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double M = sh[0];
    __syncthreads();
    double sum = 0.0;
    for (int c = threadIdx.x; c < P; c += 256) sum += exp((double)yhat[c] / tau - M);
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double S = sh[0];
    __syncthreads();
    for (int c = threadIdx.x; c < P; c += 256) q[c] = (1.0 - alpha) * exp((double)yhat[c] / tau - M) / S + alpha / P;
    __syncthreads();
    // CDF: contiguous slices per thread, then a scan of the slice totals
    const int per = (P + 255) / 256;
    const int c0 = threadIdx.x * per, c1 = min(P, c0 + per);
    double run = 0.0;
    for (int c = c0; c < c1; ++c) run += q[c];
    sh[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int t = 1; t < 256; ++t) sh[t] += sh[t - 1];
    __syncthreads();
    double base = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;
    for (int c = c0; c < c1; ++c) {
        base += q[c];
        cdf[c] = base;
    }
    __syncthreads();
    const double tot = cdf[P - 1];
    for (int k = threadIdx.x; k < K; k += 256) {
        const double x = u[k] * tot;
        int lo = 0, hi = P - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (x < cdf[mid]) hi = mid; else lo = mid + 1;
        }
        idx[k] = lo;
    }
}

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};

}  // namespace

struct fftdg_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int n_in = 0, width = 0, max_batch = 0, Bmax = 0;
    int64_t np = 0;
    bool fp32 = false;             // operands and activations FP32 (else BF16)
    Buf P, G, Mm, Vv;              // fp32 master params, grads, Adam moments
    Buf W1, W2, W3, W4, W2t, W3t;  // working copies in the operand type
    Buf A0, A0t, H1, H2, H3, H1t, H2t, Z1, Z2, Z3, y, dy, dZf, dZ, dZt, dH, gtmp, loss, idx_tmp;
    Buf pcdf;
    int64_t step = 0;
    int skip_col = -1;  // output adds skip_scale * x[skip_col] (none if < 0)
    float skip_scale = 0.f;
};

namespace {

int merr(fftdg_mlp *m, int code, const std::string &s) {
    if (m) m->err = s;
    return code;
}
#define MCHK(m, expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return merr(m, FFTDG_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int balloc(fftdg_mlp *m, Buf &b, size_t bytes) {
    if (bytes <= b.n) return FFTDG_OK;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return merr(m, FFTDG_E_NOMEM, "device allocation failed");
    }
    b.n = bytes;
    return FFTDG_OK;
}

inline unsigned nb(size_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// offsets of the flat parameter layout
struct Lay {
    int64_t W1, b1, W2, b2, W3, b3, W4, b4, n;
    Lay(int F, int H) {
        W1 = 0;
        b1 = W1 + (int64_t)H * F;
        W2 = b1 + H;
        b2 = W2 + (int64_t)H * H;
        W3 = b2 + H;
        b3 = W3 + (int64_t)H * H;
        W4 = b3 + H;
        b4 = W4 + H;
        n = b4 + 1;
    }
};

template <typename E>
int refresh_t(fftdg_mlp *m) {
    const int F = m->n_in, H = m->width;
    const Lay L(F, H);
    const float *p = (const float *)m->P.p;
    hipStream_t st = m->stream;
    hipLaunchKernelGGL(k_w_copy<E>, dim3(nb((size_t)H * KP)), dim3(256), 0, st, p + L.W1, H, F, KP, (E *)m->W1.p);
    hipLaunchKernelGGL(k_w_copy<E>, dim3(nb((size_t)H * H)), dim3(256), 0, st, p + L.W2, H, H, H, (E *)m->W2.p);
    hipLaunchKernelGGL(k_w_copy<E>, dim3(nb((size_t)H * H)), dim3(256), 0, st, p + L.W3, H, H, H, (E *)m->W3.p);
    hipLaunchKernelGGL(k_w_copy<E>, dim3(nb((size_t)H)), dim3(256), 0, st, p + L.W4, 1, H, H, (E *)m->W4.p);
    hipLaunchKernelGGL(k_transpose<E>, dim3(nb((size_t)H * H)), dim3(256), 0, st, (const E *)m->W2.p, H, H,
                       (E *)m->W2t.p);
    hipLaunchKernelGGL(k_transpose<E>, dim3(nb((size_t)H * H)), dim3(256), 0, st, (const E *)m->W3.p, H, H,
                       (E *)m->W3t.p);
    MCHK(m, hipGetLastError());
    return FFTDG_OK;
}

// the working copies of the weights from the FP32 master parameters
int refresh_w(fftdg_mlp *m) { return m->fp32 ? refresh_t<float>(m) : refresh_t<uint16_t>(m); }

template <typename E>
int gemm(fftdg_mlp *m, const E *A, int lda, const E *B, int ldb, int M, int N, int K, const float *bias, int mode,
         float *C, int ldc, E *Hh, int ldh) {
    hipLaunchKernelGGL(k_gemm<E>, dim3(N / 64, M / 64), dim3(256), 0, m->stream, A, lda, B, ldb, K, bias, mode, C,
                       ldc, Hh, ldh);
    MCHK(m, hipGetLastError());
    return FFTDG_OK;
}

// forward pass over B rows (rows of X selected by idx, or the first B rows)
template <typename E>
int forward_t(fftdg_mlp *m, const float *X, const int32_t *idx, int B, int Bp) {
    const int H = m->width;
    const Lay L(m->n_in, H);
    const float *p = (const float *)m->P.p;
    hipLaunchKernelGGL(k_gather<E>, dim3(nb((size_t)Bp * KP)), dim3(256), 0, m->stream, X, m->n_in, idx, B, Bp,
                       (E *)m->A0.p);
    int rc;
    if ((rc = gemm<E>(m, (E *)m->A0.p, KP, (E *)m->W1.p, KP, Bp, H, KP, p + L.b1, 1, (float *)m->Z1.p, H,
                      (E *)m->H1.p, H)))
        return rc;
    if ((rc = gemm<E>(m, (E *)m->H1.p, H, (E *)m->W2.p, H, Bp, H, H, p + L.b2, 1, (float *)m->Z2.p, H, (E *)m->H2.p,
                      H)))
        return rc;
    if ((rc = gemm<E>(m, (E *)m->H2.p, H, (E *)m->W3.p, H, Bp, H, H, p + L.b3, 1, (float *)m->Z3.p, H, (E *)m->H3.p,
                      H)))
        return rc;
    hipLaunchKernelGGL(k_out<E>, dim3(nb((size_t)B)), dim3(256), 0, m->stream, (const E *)m->H3.p, H,
                       (const E *)m->W4.p, p + L.b4, B, X, m->n_in, idx, m->skip_col, m->skip_scale,
                       (float *)m->y.p);
    MCHK(m, hipGetLastError());
    return FFTDG_OK;
}
int forward(fftdg_mlp *m, const float *X, const int32_t *idx, int B, int Bp) {
    return m->fp32 ? forward_t<float>(m, X, idx, B, Bp) : forward_t<uint16_t>(m, X, idx, B, Bp);
}

template <typename E>
int backward_t(fftdg_mlp *m, const float *X, const float *t, const float *w, const int32_t *idx, int B, float *g) {
    const int H = m->width, F = m->n_in;
    const int Bp = (B + 63) / 64 * 64;
    const Lay L(F, H);
    hipStream_t st = m->stream;
    int rc;
    if ((rc = forward_t<E>(m, X, idx, B, Bp))) return rc;
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, st, (const float *)m->y.p, t, w, idx, B, (float *)m->dy.p,
                       (float *)m->loss.p);
    hipLaunchKernelGGL(k_out_grad<E>, dim3(nb((size_t)H + 1)), dim3(256), 0, st, (const float *)m->dy.p,
                       (const E *)m->H3.p, H, B, g + L.W4, g + L.b4);
    // layer 3
    hipLaunchKernelGGL(k_dz<E>, dim3(nb((size_t)Bp * H)), dim3(256), 0, st, (const float *)nullptr,
                       (const float *)m->dy.p, (const E *)m->W4.p, (const float *)m->Z3.p, H, B, Bp,
                       (float *)m->dZf.p, (E *)m->dZ.p, (E *)m->dZt.p);
    hipLaunchKernelGGL(k_colsum, dim3(nb((size_t)H)), dim3(256), 0, st, (const float *)m->dZf.p, H, B, g + L.b3);
    hipLaunchKernelGGL(k_transpose<E>, dim3(nb((size_t)Bp * H)), dim3(256), 0, st, (const E *)m->H2.p, Bp, H,
                       (E *)m->H2t.p);
    if ((rc = gemm<E>(m, (E *)m->dZt.p, Bp, (E *)m->H2t.p, Bp, H, H, Bp, nullptr, 0, g + L.W3, H,
                   nullptr, 0)))
        return rc;
    if ((rc = gemm<E>(m, (E *)m->dZ.p, H, (E *)m->W3t.p, H, Bp, H, H, nullptr, 0, (float *)m->dH.p, H,
                   nullptr, 0)))
        return rc;
    // layer 2
    hipLaunchKernelGGL(k_dz<E>, dim3(nb((size_t)Bp * H)), dim3(256), 0, st, (const float *)m->dH.p,
                       (const float *)nullptr, (const E *)nullptr, (const float *)m->Z2.p, H, B, Bp,
                       (float *)m->dZf.p, (E *)m->dZ.p, (E *)m->dZt.p);
    hipLaunchKernelGGL(k_colsum, dim3(nb((size_t)H)), dim3(256), 0, st, (const float *)m->dZf.p, H, B, g + L.b2);
    hipLaunchKernelGGL(k_transpose<E>, dim3(nb((size_t)Bp * H)), dim3(256), 0, st, (const E *)m->H1.p, Bp, H,
                       (E *)m->H1t.p);
    if ((rc = gemm<E>(m, (E *)m->dZt.p, Bp, (E *)m->H1t.p, Bp, H, H, Bp, nullptr, 0, g + L.W2, H,
                   nullptr, 0)))
        return rc;
    if ((rc = gemm<E>(m, (E *)m->dZ.p, H, (E *)m->W2t.p, H, Bp, H, H, nullptr, 0, (float *)m->dH.p, H,
                   nullptr, 0)))
        return rc;
    // layer 1 (no input gradient)
    hipLaunchKernelGGL(k_dz<E>, dim3(nb((size_t)Bp * H)), dim3(256), 0, st, (const float *)m->dH.p,
                       (const float *)nullptr, (const E *)nullptr, (const float *)m->Z1.p, H, B, Bp,
                       (float *)m->dZf.p, (E *)m->dZ.p, (E *)m->dZt.p);
    hipLaunchKernelGGL(k_colsum, dim3(nb((size_t)H)), dim3(256), 0, st, (const float *)m->dZf.p, H, B, g + L.b1);
    hipLaunchKernelGGL(k_transpose<E>, dim3(nb((size_t)Bp * KP)), dim3(256), 0, st, (const E *)m->A0.p, Bp, KP,
                       (E *)m->A0t.p);
    if ((rc = gemm<E>(m, (E *)m->dZt.p, Bp, (E *)m->A0t.p, Bp, H, KP, Bp, nullptr, 0,
                   (float *)m->gtmp.p, KP, nullptr, 0)))
        return rc;
    hipLaunchKernelGGL(k_copy_cols, dim3(nb((size_t)H * F)), dim3(256), 0, st, (const float *)m->gtmp.p, H, KP, F,
                       g + L.W1);
    MCHK(m, hipGetLastError());
    return FFTDG_OK;
}
int backward(fftdg_mlp *m, const float *X, const float *t, const float *w, const int32_t *idx, int B, float *g) {
    return m->fp32 ? backward_t<float>(m, X, t, w, idx, B, g) : backward_t<uint16_t>(m, X, t, w, idx, B, g);
}

}  // namespace

extern "C" {

int fftdg_mlp_create(fftdg_mlp **out, int device, void *stream, int32_t n_in, int32_t width, int32_t max_batch) {
    return fftdg_mlp_create_ex(out, device, stream, n_in, width, max_batch, 0);
}

int fftdg_mlp_create_ex(fftdg_mlp **out, int device, void *stream, int32_t n_in, int32_t width, int32_t max_batch,
                        int32_t fp32_operands) {
    if (!out) return FFTDG_E_INVALID;
    *out = nullptr;
    if (n_in < 1 || n_in > KP || width < 64 || width % 64 || width > 1024 || max_batch < 1 || max_batch > (1 << 22) ||
        (fp32_operands != 0 && fp32_operands != 1))
        return FFTDG_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return FFTDG_E_DEVICE;
    }
    if (device < 0 || device >= ndev) return FFTDG_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        return FFTDG_E_DEVICE;
    }
    fftdg_mlp *m = new (std::nothrow) fftdg_mlp();
    if (!m) return FFTDG_E_NOMEM;
    m->device = device;
    m->stream = (hipStream_t)stream;
    m->n_in = n_in;
    m->width = width;
    m->max_batch = max_batch;
    m->fp32 = fp32_operands != 0;
    m->Bmax = (max_batch + 63) / 64 * 64;
    const Lay L(n_in, width);
    m->np = L.n;
    const size_t H = width, Bm = m->Bmax;
    int rc = 0;
    Buf *f32n[] = {&m->P, &m->G, &m->Mm, &m->Vv};
    for (Buf *b : f32n)
        if (!rc) rc = balloc(m, *b, sizeof(float) * L.n);
    const size_t bf = m->fp32 ? sizeof(float) : sizeof(uint16_t);  // operand element
    if (!rc) rc = balloc(m, m->W1, bf * H * KP);
    if (!rc) rc = balloc(m, m->W2, bf * H * H);
    if (!rc) rc = balloc(m, m->W3, bf * H * H);
    if (!rc) rc = balloc(m, m->W4, bf * H);
    if (!rc) rc = balloc(m, m->W2t, bf * H * H);
    if (!rc) rc = balloc(m, m->W3t, bf * H * H);
    if (!rc) rc = balloc(m, m->A0, bf * Bm * KP);
    if (!rc) rc = balloc(m, m->A0t, bf * Bm * KP);
    Buf *hb[] = {&m->H1, &m->H2, &m->H3, &m->H1t, &m->H2t, &m->dZ, &m->dZt};
    for (Buf *b : hb)
        if (!rc) rc = balloc(m, *b, bf * Bm * H);
    Buf *zb[] = {&m->Z1, &m->Z2, &m->Z3, &m->dZf, &m->dH};
    for (Buf *b : zb)
        if (!rc) rc = balloc(m, *b, sizeof(float) * Bm * H);
    if (!rc) rc = balloc(m, m->y, sizeof(float) * Bm);
    if (!rc) rc = balloc(m, m->dy, sizeof(float) * Bm);
    if (!rc) rc = balloc(m, m->gtmp, sizeof(float) * H * KP);
    if (!rc) rc = balloc(m, m->loss, sizeof(float) * 4);
    if (rc) {
        fftdg_mlp_destroy(m);
        return rc;
    }
    std::vector<float> zero(L.n, 0.f);
    if (hipMemcpy(m->P.p, zero.data(), sizeof(float) * L.n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->Mm.p, zero.data(), sizeof(float) * L.n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->Vv.p, zero.data(), sizeof(float) * L.n, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        fftdg_mlp_destroy(m);
        return FFTDG_E_DEVICE;
    }
    if ((rc = refresh_w(m)) || hipStreamSynchronize(m->stream) != hipSuccess) {
        fftdg_mlp_destroy(m);
        return rc ? rc : FFTDG_E_DEVICE;
    }
    *out = m;
    return FFTDG_OK;
}

void fftdg_mlp_destroy(fftdg_mlp *m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipStreamSynchronize(m->stream);
    Buf *all[] = {&m->P,   &m->G,   &m->Mm,  &m->Vv,  &m->W1,  &m->W2,  &m->W3, &m->W4,  &m->W2t, &m->W3t,
                  &m->A0,  &m->A0t, &m->H1,  &m->H2,  &m->H3,  &m->H1t, &m->H2t, &m->Z1, &m->Z2,  &m->Z3,
                  &m->y,   &m->dy,  &m->dZf, &m->dZ,  &m->dZt, &m->dH,  &m->gtmp, &m->loss, &m->idx_tmp, &m->pcdf};
    for (Buf *b : all)
        if (b->p) (void)hipFree(b->p);
    delete m;
}

const char *fftdg_mlp_last_error(const fftdg_mlp *m) { return m ? m->err.c_str() : "network is NULL"; }

int64_t fftdg_mlp_num_params(const fftdg_mlp *m) { return m ? m->np : -1; }

int fftdg_mlp_set_params(fftdg_mlp *m, const float *p_host, int64_t n) {
    if (!m) return FFTDG_E_INVALID;
    if (!p_host || n != m->np) return merr(m, FFTDG_E_INVALID, "set_params: wrong size or NULL");
    MCHK(m, hipSetDevice(m->device));
    MCHK(m, hipMemcpyAsync(m->P.p, p_host, sizeof(float) * n, hipMemcpyHostToDevice, m->stream));
    std::vector<float> zero(n, 0.f);
    MCHK(m, hipMemcpyAsync(m->Mm.p, zero.data(), sizeof(float) * n, hipMemcpyHostToDevice, m->stream));
    MCHK(m, hipMemcpyAsync(m->Vv.p, zero.data(), sizeof(float) * n, hipMemcpyHostToDevice, m->stream));
    m->step = 0;
    int rc = refresh_w(m);
    if (rc) return rc;
    MCHK(m, hipStreamSynchronize(m->stream));
    return FFTDG_OK;
}

int fftdg_mlp_get_params(fftdg_mlp *m, float *p_host, int64_t n) {
    if (!m) return FFTDG_E_INVALID;
    if (!p_host || n != m->np) return merr(m, FFTDG_E_INVALID, "get_params: wrong size or NULL");
    MCHK(m, hipSetDevice(m->device));
    MCHK(m, hipMemcpyAsync(p_host, m->P.p, sizeof(float) * n, hipMemcpyDeviceToHost, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
    return FFTDG_OK;
}

int fftdg_mlp_set_skip(fftdg_mlp *m, int32_t col, float scale) {
    if (!m) return FFTDG_E_INVALID;
    if (col < -1 || col >= m->n_in || !std::isfinite(scale))
        return merr(m, FFTDG_E_INVALID, "set_skip: column out of range or non-finite scale");
    m->skip_col = col;
    m->skip_scale = col >= 0 ? scale : 0.f;
    return FFTDG_OK;
}

int fftdg_mlp_forward(fftdg_mlp *m, const float *x, int32_t n, float *y) {
    if (!m) return FFTDG_E_INVALID;
    if (!x || !y || n < 0) return merr(m, FFTDG_E_INVALID, "forward: NULL pointer or negative size");
    MCHK(m, hipSetDevice(m->device));
    for (int32_t b0 = 0; b0 < n; b0 += m->max_batch) {
        const int B = std::min(m->max_batch, n - b0), Bp = (B + 63) / 64 * 64;
        int rc = forward(m, x + (size_t)b0 * m->n_in, nullptr, B, Bp);
        if (rc) return rc;
        MCHK(m, hipMemcpyAsync(y + b0, m->y.p, sizeof(float) * B, hipMemcpyDeviceToDevice, m->stream));
    }
    return FFTDG_OK;
}

int fftdg_mlp_grad(fftdg_mlp *m, const float *x_all, const float *t_all, const float *w_all, const int32_t *idx,
                   int32_t B, float *grad, float *loss_host) {
    if (!m) return FFTDG_E_INVALID;
    if (!x_all || !t_all || !w_all || !grad || B < 1 || B > m->max_batch)
        return merr(m, FFTDG_E_INVALID, "grad: NULL pointer or batch size outside 1..max_batch");
    MCHK(m, hipSetDevice(m->device));
    int rc = backward(m, x_all, t_all, w_all, idx, B, grad);
    if (rc) return rc;
    if (loss_host) {
        MCHK(m, hipMemcpyAsync(loss_host, m->loss.p, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
    }
    return FFTDG_OK;
}

int fftdg_mlp_train_step(fftdg_mlp *m, const float *x_all, const float *t_all, const float *w_all,
                         const int32_t *idx, int32_t B, float lr, float *loss_host) {
    if (!m) return FFTDG_E_INVALID;
    if (!(lr > 0.f) || !std::isfinite(lr)) return merr(m, FFTDG_E_INVALID, "train_step: learning rate must be > 0");
    int rc = fftdg_mlp_grad(m, x_all, t_all, w_all, idx, B, (float *)m->G.p, nullptr);
    if (rc) return rc;
    ++m->step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)m->step), c2 = 1.f - powf(b2, (float)m->step);
    hipLaunchKernelGGL(k_adam, dim3(nb((size_t)m->np)), dim3(256), 0, m->stream, (float *)m->P.p,
                       (const float *)m->G.p, (float *)m->Mm.p, (float *)m->Vv.p, (int)m->np, lr, b1, b2, 1e-8f, c1,
                       c2);
    MCHK(m, hipGetLastError());
    if ((rc = refresh_w(m))) return rc;
    if (loss_host) {
        MCHK(m, hipMemcpyAsync(loss_host, m->loss.p, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
    }
    return FFTDG_OK;
}

int fftdg_proposal_sample(fftdg_mlp *m, const float *yhat, int32_t P, double alpha, double tau, int32_t K,
                          const double *u, int32_t *idx, double *q) {
    if (!m) return FFTDG_E_INVALID;
    if (!yhat || !u || !idx || !q || P < 1 || K < 0)
        return merr(m, FFTDG_E_INVALID, "proposal_sample: NULL pointer or bad size");
    if (!(alpha >= 0.0 && alpha <= 1.0) || !(tau > 0.0) || !std::isfinite(tau))
        return merr(m, FFTDG_E_INVALID, "proposal_sample: need 0 <= alpha <= 1 and tau > 0");
    MCHK(m, hipSetDevice(m->device));
    if (m->pcdf.n < sizeof(double) * (size_t)P) {
        if (m->pcdf.p) (void)hipFree(m->pcdf.p);
        m->pcdf.p = nullptr;
        m->pcdf.n = 0;
        if (hipMalloc(&m->pcdf.p, sizeof(double) * (size_t)P) != hipSuccess) {
            (void)hipGetLastError();
            return merr(m, FFTDG_E_NOMEM, "proposal_sample: allocation failed");
        }
        m->pcdf.n = sizeof(double) * (size_t)P;
    }
    hipLaunchKernelGGL(k_proposal, dim3(1), dim3(256), 0, m->stream, yhat, P, alpha, tau, K, u, idx, q,
                       (double *)m->pcdf.p);
    MCHK(m, hipGetLastError());
    return FFTDG_OK;
}

}  // extern "C"
