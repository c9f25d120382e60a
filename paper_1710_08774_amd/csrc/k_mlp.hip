// Training and inference kernels of the tuning cost model: a multilayer
// perceptron with three ReLU hidden layers of width H and one linear output,
// FP32, trained on mean squared error with Adam.  Parameters are one flat
// array: W1 (H,d) b1 (H) W2 (H,H) b2 (H) W3 (H,H) b3 (H) W4 (1,H) b4 (1),
// weights row-major W[out][in].
//
// The contractions are small (batches of a few thousand samples, width 64),
// so one LDS-tiled FP32 GEMM kernel with transpose flags serves the forward
// products and both backward products; the rest are elementwise kernels.
#include <hip/hip_runtime.h>

#include "../../include/hfav_mlp.h"

namespace {

constexpr int TS = 16;

// C[M,N] = op(A)[M,K] * op(B)[K,N] (+ C if acc); op(X) = X or X^T
// (transposed operands are stored row-major as their untransposed shape).
__global__ __launch_bounds__(TS * TS) void gemm_kernel(const float *A, const float *B, float *C, int M, int N,
                                                       int K, int ta, int tb, int acc) {
    __shared__ float sa[TS][TS + 1];
    __shared__ float sb[TS][TS + 1];
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    const int row = blockIdx.y * TS + ty, col = blockIdx.x * TS + tx;
    float sum = 0.f;
    for (int k0 = 0; k0 < K; k0 += TS) {
        // A tile: rows row-block, cols k0..k0+TS
        const int ak = k0 + tx, ar = blockIdx.y * TS + ty;
        float av = 0.f;
        if (ar < M && ak < K) av = ta ? A[(size_t)ak * M + ar] : A[(size_t)ar * K + ak];
        sa[ty][tx] = av;
        const int bk = k0 + ty, bc = blockIdx.x * TS + tx;
        float bv = 0.f;
        if (bk < K && bc < N) bv = tb ? B[(size_t)bc * K + bk] : B[(size_t)bk * N + bc];
        sb[ty][tx] = bv;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TS; ++q) sum = fmaf(sa[ty][q], sb[q][tx], sum);
        __syncthreads();
    }
    if (row < M && col < N) {
        float *c = C + (size_t)row * N + col;
        *c = acc ? *c + sum : sum;
    }
}

// Z[M,N] += b (per column); ReLU in place when relu
__global__ void bias_act_kernel(float *Z, const float *b, int M, int N, int relu) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)M * N) return;
    float v = Z[q] + b[q % N];
    Z[q] = relu ? fmaxf(v, 0.f) : v;
}

// dZ = dH where H > 0, else 0 (in place on dH)
__global__ void relu_bwd_kernel(float *dH, const float *H, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n && !(H[q] > 0.f)) dH[q] = 0.f;
}

// db[n] = sum over rows of dZ[:, n]
__global__ void colsum_kernel(const float *dZ, float *db, int M, int N) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    float s = 0.f;
    for (int r = 0; r < M; ++r) s += dZ[(size_t)r * N + c];
    db[c] = s;
}

// dy = 2 (y - t) / M; loss = mean (y - t)^2 (single workgroup)
__global__ __launch_bounds__(256) void loss_kernel(const float *y, const float *t, float *dy, float *loss, int M) {
    __shared__ float red[256];
    float s = 0.f;
    for (int q = threadIdx.x; q < M; q += 256) {
        const float r = y[q] - t[q];
        dy[q] = 2.f * r / (float)M;
        s += r * r;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = red[0] / (float)M;
}

__global__ void adam_kernel(float *P, const float *G, float *m, float *v, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float g = G[q];
    const float mq = b1 * m[q] + (1.f - b1) * g;
    const float vq = b2 * v[q] + (1.f - b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    P[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

struct Layout {
    const float *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
};
struct GLayout {
    float *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
};
template <class P, class L>
L layout(P base, int d, int H) {
    L l;
    l.W1 = base;
    l.b1 = l.W1 + (size_t)H * d;
    l.W2 = l.b1 + H;
    l.b2 = l.W2 + (size_t)H * H;
    l.W3 = l.b2 + H;
    l.b3 = l.W3 + (size_t)H * H;
    l.W4 = l.b3 + H;
    l.b4 = l.W4 + H;
    return l;
}

void gemm(const float *A, const float *B, float *C, int M, int N, int K, int ta, int tb, int acc, hipStream_t s) {
    dim3 grid((N + TS - 1) / TS, (M + TS - 1) / TS);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(TS * TS), 0, s, A, B, C, M, N, K, ta, tb, acc);
}
void bias_act(float *Z, const float *b, int M, int N, int relu, hipStream_t s) {
    const size_t n = (size_t)M * N;
    hipLaunchKernelGGL(bias_act_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Z, b, M, N, relu);
}

int status(hipError_t e) { return e == hipSuccess ? 0 : 8; }

// forward into the workspace: H1, H2, H3 (n,H) and y (n)
void forward(const float *X, int n, int d, int H, const float *Pp, float *ws, float *y, hipStream_t s) {
    const Layout P = layout<const float *, Layout>(Pp, d, H);
    float *H1 = ws, *H2 = H1 + (size_t)n * H, *H3 = H2 + (size_t)n * H;
    gemm(X, P.W1, H1, n, H, d, 0, 1, 0, s);
    bias_act(H1, P.b1, n, H, 1, s);
    gemm(H1, P.W2, H2, n, H, H, 0, 1, 0, s);
    bias_act(H2, P.b2, n, H, 1, s);
    gemm(H2, P.W3, H3, n, H, H, 0, 1, 0, s);
    bias_act(H3, P.b3, n, H, 1, s);
    gemm(H3, P.W4, y, n, 1, H, 0, 1, 0, s);
    bias_act(y, P.b4, n, 1, 0, s);
}

}  // namespace

extern "C" size_t hfav_mlp_workspace_bytes(int n, int d, int H) {
    (void)d;
    return sizeof(float) * ((size_t)5 * n * H + 2 * (size_t)n);
}

extern "C" size_t hfav_mlp_nparams(int d, int H) {
    return (size_t)H * d + H + 2 * ((size_t)H * H + H) + H + 1;
}

extern "C" int hfav_mlp_forward(const float *X, int n, int d, int H, const float *params, float *y,
                                void *workspace, void *stream) {
    if (!X || !params || !y || !workspace || n < 1 || d < 1 || H < 1) return 1;
    forward(X, n, d, H, params, (float *)workspace, y, (hipStream_t)stream);
    return status(hipGetLastError());
}

extern "C" int hfav_mlp_loss_grad(const float *X, const float *t, int n, int d, int H, const float *params,
                                  float *grads, float *loss, void *workspace, void *stream) {
    if (!X || !t || !params || !grads || !workspace || n < 1 || d < 1 || H < 1) return 1;
    hipStream_t s = (hipStream_t)stream;
    float *ws = (float *)workspace;
    float *H1 = ws, *H2 = H1 + (size_t)n * H, *H3 = H2 + (size_t)n * H;
    float *dA = H3 + (size_t)n * H, *dB = dA + (size_t)n * H;
    float *y = dB + (size_t)n * H, *dy = y + n;
    forward(X, n, d, H, params, ws, y, s);
    const Layout P = layout<const float *, Layout>(params, d, H);
    const GLayout G = layout<float *, GLayout>(grads, d, H);
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, y, t, dy, loss, n);
    // output layer
    gemm(dy, H3, G.W4, 1, H, n, 1, 0, 0, s);                 // gW4 = dy^T H3
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(64), 0, s, dy, G.b4, n, 1);
    gemm(dy, P.W4, dA, n, H, 1, 0, 0, 0, s);                  // dH3 = dy W4
    hipLaunchKernelGGL(relu_bwd_kernel, dim3((unsigned)(((size_t)n * H + 255) / 256)), dim3(256), 0, s, dA, H3,
                       (size_t)n * H);
    // layer 3
    gemm(dA, H2, G.W3, H, H, n, 1, 0, 0, s);                  // gW3 = dZ3^T H2
    hipLaunchKernelGGL(colsum_kernel, dim3((H + 63) / 64), dim3(64), 0, s, dA, G.b3, n, H);
    gemm(dA, P.W3, dB, n, H, H, 0, 0, 0, s);                  // dH2 = dZ3 W3
    hipLaunchKernelGGL(relu_bwd_kernel, dim3((unsigned)(((size_t)n * H + 255) / 256)), dim3(256), 0, s, dB, H2,
                       (size_t)n * H);
    // layer 2
    gemm(dB, H1, G.W2, H, H, n, 1, 0, 0, s);
    hipLaunchKernelGGL(colsum_kernel, dim3((H + 63) / 64), dim3(64), 0, s, dB, G.b2, n, H);
    gemm(dB, P.W2, dA, n, H, H, 0, 0, 0, s);                  // dH1 = dZ2 W2
    hipLaunchKernelGGL(relu_bwd_kernel, dim3((unsigned)(((size_t)n * H + 255) / 256)), dim3(256), 0, s, dA, H1,
                       (size_t)n * H);
    // layer 1
    gemm(dA, X, G.W1, H, d, n, 1, 0, 0, s);                   // gW1 = dZ1^T X
    hipLaunchKernelGGL(colsum_kernel, dim3((H + 63) / 64), dim3(64), 0, s, dA, G.b1, n, H);
    return status(hipGetLastError());
}

extern "C" int hfav_mlp_adam(float *params, const float *grads, float *m, float *v, int np, float lr, float b1,
                             float b2, float eps, int step, void *stream) {
    if (!params || !grads || !m || !v || np < 1 || step < 1) return 1;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((np + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grads, m, v,
                       np, lr, b1, b2, eps, c1, c2);
    return status(hipGetLastError());
}
