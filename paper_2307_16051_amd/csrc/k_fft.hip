// k_fft.hip -- FP64 FFT and the O(N log N) H-equation operators.
//
// In eq. (3.2) the sum sum_j x_j mu_i / (mu_i + mu_j) equals (i + 1/2) S_i
// with S_i = sum_j h_{i+j} x_j, h_k = 1/(k+1) (0-based, mu_i = (i + 1/2)/N):
// a Hankel product.  With y the reversed x (y_m = x_{N-1-m}), S_i is entry
// i + N - 1 of the linear convolution h * y, which a cyclic convolution of
// length L >= 2N - 1 reproduces exactly on those entries.  So the residual
// F(x), and the Jacobian-vector product J v = v - diag(1/D^2) K v of the same
// operator, cost two FFTs of length L each (the transform of h is kept),
// instead of N^2 terms -- the cost model the paper states for this example
// (Section 3).
//
// FFT: complex FP64, L = 2^p (2 <= L <= 65536), four-step: L = n1 n2,
//   X[k2 + n2 k1] = sum_j1 W_n1^(j1 k1) W_L^(j1 k2) sum_j2 x[j1 + n1 j2] W_n2^(j2 k2),
// pass A: n1 transforms of length n2 (one per j1), times the twiddle W_L^(j1 k2);
// pass B: n2 transforms of length n1 (one per k2).  Each workgroup transforms
// R = 16 sequences in LDS (iterative radix-2 with bit-reversed loading), which
// keeps the global reads and writes in 16-element runs.  Twiddles come from a
// table tw[k] = exp(-2 pi i k / L) computed once with sincospi (FP64).
#include <hip/hip_runtime.h>

#include "n3p_internal.hpp"

namespace n3p {

constexpr int FFT_R = 16;             // sequences per workgroup
constexpr int FFT_MAXM = 256;         // largest sub-transform length (L <= 65536)
constexpr int FFT_THREADS = 256;

typedef double2 cplx;

__device__ __forceinline__ cplx cmul(cplx a, cplx b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void k_fft_twiddles(int L, cplx *tw)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < L) {
        double s, c;
        sincospi(-2.0 * (double)k / (double)L, &s, &c);
        tw[k] = make_double2(c, s);
    }
}

__device__ __forceinline__ int bitrev(int v, int bits)
{
    return bits ? (int)(__brev((unsigned)v) >> (32 - bits)) : 0;
}

// In-LDS radix-2 transforms of `rows` sequences of length m (buf[r][.],
// loaded in bit-reversed order).  W_m^t = tw[t * (L / m)].
__device__ __forceinline__ void lds_fft(cplx (*buf)[FFT_MAXM + 1], int rows, int m, int logm,
                                        const cplx *__restrict__ tw, int L)
{
    const int t = threadIdx.x;
    const int nbf = rows * (m >> 1);
    for (int s = 0; s < logm; ++s) {
        const int half = 1 << s, stride = L / (half << 1);
        for (int e = t; e < nbf; e += FFT_THREADS) {
            const int r = e / (m >> 1), b = e % (m >> 1);
            const int grp = b / half, pos = b % half;
            const int i0 = grp * (half << 1) + pos, i1 = i0 + half;
            const cplx w = tw[pos * stride];
            const cplx u = buf[r][i0], v = cmul(buf[r][i1], w);
            buf[r][i0] = make_double2(u.x + v.x, u.y + v.y);
            buf[r][i1] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// Pass A: for j1 in this block's rows, transform x[j1 + n1 j2] over j2
// (length n2), multiply by W_L^(j1 k2), store A[j1 * n2 + k2].
__global__ __launch_bounds__(FFT_THREADS) void k_fft_pass_a(int L, int n1, int n2, int logn2,
                                                            const cplx *__restrict__ x,
                                                            const cplx *__restrict__ tw,
                                                            cplx *__restrict__ A)
{
    __shared__ cplx buf[FFT_R][FFT_MAXM + 1];
    const int R = n1 < FFT_R ? n1 : FFT_R;
    const int j1b = blockIdx.x * R, t = threadIdx.x;
    for (int e = t; e < R * n2; e += FFT_THREADS) {  // e = r + R j2: runs of R along j1
        const int r = e % R, j2 = e / R;
        buf[r][bitrev(j2, logn2)] = x[(j1b + r) + (int64_t)n1 * j2];
    }
    __syncthreads();
    lds_fft(buf, R, n2, logn2, tw, L);
    for (int e = t; e < R * n2; e += FFT_THREADS) {
        const int r = e / n2, k2 = e % n2;
        const int j1 = j1b + r;
        A[(int64_t)j1 * n2 + k2] = cmul(buf[r][k2], tw[(int)(((int64_t)j1 * k2) % L)]);
    }
}

// Pass B: for k2 in this block's columns, transform A[j1 * n2 + k2] over j1
// (length n1), store X[k2 + n2 k1].
__global__ __launch_bounds__(FFT_THREADS) void k_fft_pass_b(int L, int n1, int n2, int logn1,
                                                            const cplx *__restrict__ A,
                                                            const cplx *__restrict__ tw,
                                                            cplx *__restrict__ X)
{
    __shared__ cplx buf[FFT_R][FFT_MAXM + 1];
    const int R = n2 < FFT_R ? n2 : FFT_R;
    const int k2b = blockIdx.x * R, t = threadIdx.x;
    for (int e = t; e < R * n1; e += FFT_THREADS) {  // runs of R along k2
        const int r = e % R, j1 = e / R;
        buf[r][bitrev(j1, logn1)] = A[(int64_t)j1 * n2 + k2b + r];
    }
    __syncthreads();
    lds_fft(buf, R, n1, logn1, tw, L);
    for (int e = t; e < R * n1; e += FFT_THREADS) {
        const int r = e % R, k1 = e / R;
        X[(k2b + r) + (int64_t)n2 * k1] = buf[r][k1];
    }
}

// ------------------------------------------------------------ Hankel pieces
// y = reversed x (or v), zero padded, as complex
__global__ void k_hk_pack_rev(int64_t n, int L, const double *__restrict__ v, cplx *__restrict__ y)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < L) y[m] = make_double2(m < n ? v[n - 1 - m] : 0.0, 0.0);
}
__global__ void k_hk_pack_rev_f32(int64_t n, int L, const float *__restrict__ v, cplx *__restrict__ y)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < L) y[m] = make_double2(m < n ? (double)v[n - 1 - m] : 0.0, 0.0);
}
// h_k = 1/(k+1) for k < 2n - 1, zero beyond
__global__ void k_hk_pack_h(int64_t n, int L, cplx *__restrict__ y)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < L) y[k] = make_double2(k < 2 * n - 1 ? 1.0 / (double)(k + 1) : 0.0, 0.0);
}
// Z = conj(Y . H): the inverse transform is conj(FFT(conj(.))) / L
__global__ void k_hk_mul_conj(int L, const cplx *__restrict__ Y, const cplx *__restrict__ H,
                              cplx *__restrict__ Z)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < L) {
        const cplx p = cmul(Y[k], H[k]);
        Z[k] = make_double2(p.x, -p.y);
    }
}
// S_i = Re(IFFT)[i + n - 1] = Re(conj(W))[i + n - 1] / L with W = FFT(Z)
__device__ __forceinline__ double hk_sum(const cplx *__restrict__ W, int64_t n, int L, int64_t i)
{
    return W[i + n - 1].x / (double)L;
}
__global__ void k_hk_residual(int64_t n, int L, double c, const double *__restrict__ x,
                              const cplx *__restrict__ W, double *__restrict__ F,
                              double *__restrict__ D)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double d = 1.0 - c / (2.0 * (double)n) * ((double)i + 0.5) * hk_sum(W, n, L, i);
        if (D) D[i] = d;
        F[i] = x[i] - 1.0 / d;
    }
}
// y = J v = v - (c/(2N)) (i + 1/2) S_i(v) / D_i^2, written FP32 (or r = b - J v)
__global__ void k_hk_jv(int64_t n, int64_t np, int L, double c, const double *__restrict__ D,
                        const float *__restrict__ v, const cplx *__restrict__ W,
                        const float *__restrict__ b, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double d = D[i];
        const double jv = (double)v[i] - c / (2.0 * (double)n) * ((double)i + 0.5) *
                                             hk_sum(W, n, L, i) / (d * d);
        out[i] = b ? (float)((double)b[i] - jv) : (float)jv;
    } else if (i < np) {
        out[i] = 0.0f;
    }
}

// ------------------------------------------------------------------ plans
int fft_length(int64_t n)
{
    int64_t L = 2;
    while (L < 2 * n - 1) L <<= 1;
    return L <= 65536 ? (int)L : 0;
}

static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

static int ilog2(int v)
{
    int p = 0;
    while ((1 << p) < v) ++p;
    return p;
}

// X = FFT(x), length L; A is scratch of L entries
hipError_t launch_fft(int L, const cplx *x, cplx *A, cplx *X, const cplx *tw, hipStream_t s)
{
    const int p = ilog2(L), p1 = p / 2, p2 = p - p1;
    const int n1 = 1 << p1, n2 = 1 << p2;
    const int Ra = n1 < FFT_R ? n1 : FFT_R, Rb = n2 < FFT_R ? n2 : FFT_R;
    hipLaunchKernelGGL(k_fft_pass_a, dim3(n1 / Ra), dim3(FFT_THREADS), 0, s, L, n1, n2, p2, x, tw, A);
    hipLaunchKernelGGL(k_fft_pass_b, dim3(n2 / Rb), dim3(FFT_THREADS), 0, s, L, n1, n2, p1, A, tw, X);
    return hipGetLastError();
}

// One-time set-up for size n: twiddles and the transform of h.
hipError_t launch_hk_setup(int64_t n, int L, cplx *tw, cplx *H, cplx *t1, cplx *t2, hipStream_t s)
{
    hipLaunchKernelGGL(k_fft_twiddles, dim3(nb(L, 256)), dim3(256), 0, s, L, tw);
    hipLaunchKernelGGL(k_hk_pack_h, dim3(nb(L, 256)), dim3(256), 0, s, n, L, t1);
    return launch_fft(L, t1, t2, H, tw, s);
}

// W such that S_i(v) = Re W[i + n - 1] / L; v FP64 (v64) or FP32 (v32)
static hipError_t hankel(int64_t n, int L, const double *v64, const float *v32, const cplx *tw,
                         const cplx *H, cplx *t1, cplx *t2, cplx *W, hipStream_t s)
{
    if (v64) hipLaunchKernelGGL(k_hk_pack_rev, dim3(nb(L, 256)), dim3(256), 0, s, n, L, v64, t1);
    else hipLaunchKernelGGL(k_hk_pack_rev_f32, dim3(nb(L, 256)), dim3(256), 0, s, n, L, v32, t1);
    hipError_t e = launch_fft(L, t1, t2, W, tw, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hk_mul_conj, dim3(nb(L, 256)), dim3(256), 0, s, L, W, H, t1);
    return launch_fft(L, t1, t2, W, tw, s);
}

hipError_t launch_hk_residual(int64_t n, int L, double c, const double *x, const cplx *tw,
                              const cplx *H, cplx *t1, cplx *t2, cplx *W, double *F, double *D,
                              hipStream_t s)
{
    hipError_t e = hankel(n, L, x, nullptr, tw, H, t1, t2, W, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hk_residual, dim3(nb(n, 256)), dim3(256), 0, s, n, L, c, x, W, F, D);
    return hipGetLastError();
}

hipError_t launch_hk_jv(int64_t n, int64_t np, int L, double c, const double *D, const float *v,
                        const float *b, float *out, const cplx *tw, const cplx *H, cplx *t1,
                        cplx *t2, cplx *W, hipStream_t s)
{
    hipError_t e = hankel(n, L, nullptr, v, tw, H, t1, t2, W, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hk_jv, dim3(nb(np, 256)), dim3(256), 0, s, n, np, L, c, D, v, W, b, out);
    return hipGetLastError();
}

}  // namespace n3p
