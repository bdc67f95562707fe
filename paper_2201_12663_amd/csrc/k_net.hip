// Rank-proposal network: a small FP32 multilayer perceptron
//     x (67) -> relu(W1 x + b1) (128) -> relu(W2 h1 + b2) (128) -> W3 h2 + b3 (2)
// with its forward pass, the gradient of the mean-squared-error loss
//     L = 1/(2B) sum_b sum_o (y_bo - t_bo)^2
// by back-propagation, and Adam updates.  Rows of X, H, Y are samples
// (row-major); W_l is (out x in), row-major.  Every reduction over the batch
// runs in a fixed order, so a training step is bitwise repeatable.
//
// Parameter vector (floats): W1 | b1 | W2 | b2 | W3 | b3.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int NI = NET_IN, NH = NET_HID, NO = NET_OUT;

// Z = X W^T + b (B x out); H = relu(Z) when relu, else H = Z
__global__ __launch_bounds__(256) void k_fwd(int B, int in, int out, const float* __restrict__ X,
                                             const float* __restrict__ W, const float* __restrict__ b,
                                             float* __restrict__ Z, float* __restrict__ H, int relu) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)B * out) return;
    const int s = (int)(e / out), o = (int)(e % out);
    const float* x = X + (int64_t)s * in;
    const float* w = W + (int64_t)o * in;
    float acc = b[o];
    for (int i = 0; i < in; ++i) acc = fmaf(x[i], w[i], acc);
    if (Z) Z[e] = acc;
    H[e] = relu ? fmaxf(acc, 0.0f) : acc;
}

// dY = (Y - T) / B and the per-sample loss terms (summed in fixed order by k_loss)
__global__ void k_out_grad(int B, const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY,
                           float* __restrict__ lterm) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float l = 0.0f;
    for (int o = 0; o < NO; ++o) {
        const float d = Y[s * NO + o] - T[s * NO + o];
        dY[s * NO + o] = d / (float)B;
        l += d * d;
    }
    lterm[s] = 0.5f * l;
}

__global__ __launch_bounds__(256) void k_loss(int B, const float* __restrict__ lterm, float* __restrict__ loss) {
    __shared__ float red[256];
    float acc = 0.0f;
    for (int s = threadIdx.x; s < B; s += 256) acc += lterm[s];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)B;
}

// dHprev = dZ W (B x in), masked by the previous pre-activation: dZprev = dHprev * (Zprev > 0)
__global__ __launch_bounds__(256) void k_bwd_input(int B, int in, int out, const float* __restrict__ dZ,
                                                   const float* __restrict__ W, const float* __restrict__ Zprev,
                                                   float* __restrict__ dZprev) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)B * in) return;
    const int s = (int)(e / in), i = (int)(e % in);
    const float* dz = dZ + (int64_t)s * out;
    float acc = 0.0f;
    for (int o = 0; o < out; ++o) acc = fmaf(dz[o], W[(int64_t)o * in + i], acc);
    dZprev[e] = (Zprev[e] > 0.0f) ? acc : 0.0f;
}

// dW = dZ^T Hprev (out x in), db = sum_s dZ (one thread per weight; bias by i == in)
__global__ __launch_bounds__(256) void k_bwd_weight(int B, int in, int out, const float* __restrict__ dZ,
                                                    const float* __restrict__ Hprev, float* __restrict__ dW,
                                                    float* __restrict__ db) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)out * (in + 1)) return;
    const int o = (int)(e / (in + 1)), i = (int)(e % (in + 1));
    float acc = 0.0f;
    if (i < in) {
        for (int s = 0; s < B; ++s) acc = fmaf(dZ[(int64_t)s * out + o], Hprev[(int64_t)s * in + i], acc);
        dW[(int64_t)o * in + i] = acc;
    } else {
        for (int s = 0; s < B; ++s) acc += dZ[(int64_t)s * out + o];
        db[o] = acc;
    }
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t net_work_floats(int B) {
    // Z1 H1 Z2 H2 (B x NH each), Y dY (B x NO), loss terms (B), dZ1 dZ2 (B x NH)
    return (size_t)B * (6 * NH + 2 * NO + 1) + 64;
}

hipError_t net_forward(const float* P, int B, const float* X, float* Y, float* work, hipStream_t st) {
    const float *W1 = P, *b1 = W1 + NH * NI, *W2 = b1 + NH, *b2 = W2 + NH * NH, *W3 = b2 + NH, *b3 = W3 + NO * NH;
    float* Z1 = work;
    float* H1 = Z1 + (size_t)B * NH;
    float* Z2 = H1 + (size_t)B * NH;
    float* H2 = Z2 + (size_t)B * NH;
    hipLaunchKernelGGL(k_fwd, dim3(blocks((int64_t)B * NH)), dim3(256), 0, st, B, NI, NH, X, W1, b1, Z1, H1, 1);
    hipLaunchKernelGGL(k_fwd, dim3(blocks((int64_t)B * NH)), dim3(256), 0, st, B, NH, NH, H1, W2, b2, Z2, H2, 1);
    hipLaunchKernelGGL(k_fwd, dim3(blocks((int64_t)B * NO)), dim3(256), 0, st, B, NH, NO, H2, W3, b3, nullptr, Y, 0);
    return hipGetLastError();
}

hipError_t net_train_step(float* P, float* G, float* Madam, float* Vadam, int step, float lr, int B, const float* X,
                          const float* T, float* loss, float* work, hipStream_t st) {
    hipError_t e;
    float* Z1 = work;
    float* H1 = Z1 + (size_t)B * NH;
    float* Z2 = H1 + (size_t)B * NH;
    float* H2 = Z2 + (size_t)B * NH;
    float* Y = H2 + (size_t)B * NH;
    float* dY = Y + (size_t)B * NO;
    float* lt = dY + (size_t)B * NO;
    float* dZ2 = lt + B;
    float* dZ1 = dZ2 + (size_t)B * NH;
    if ((e = net_forward(P, B, X, Y, work, st)) != hipSuccess) return e;
    const float *W2 = P + NH * NI + NH, *W3 = W2 + NH * NH + NH;
    float *gW1 = G, *gb1 = gW1 + NH * NI, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH, *gW3 = gb2 + NH, *gb3 = gW3 + NO * NH;
    hipLaunchKernelGGL(k_out_grad, dim3(blocks(B)), dim3(256), 0, st, B, Y, T, dY, lt);
    if (loss) hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, st, B, lt, loss);
    // layer 3
    hipLaunchKernelGGL(k_bwd_weight, dim3(blocks((int64_t)NO * (NH + 1))), dim3(256), 0, st, B, NH, NO, dY, H2, gW3, gb3);
    hipLaunchKernelGGL(k_bwd_input, dim3(blocks((int64_t)B * NH)), dim3(256), 0, st, B, NH, NO, dY, W3, Z2, dZ2);
    // layer 2
    hipLaunchKernelGGL(k_bwd_weight, dim3(blocks((int64_t)NH * (NH + 1))), dim3(256), 0, st, B, NH, NH, dZ2, H1, gW2, gb2);
    hipLaunchKernelGGL(k_bwd_input, dim3(blocks((int64_t)B * NH)), dim3(256), 0, st, B, NH, NH, dZ2, W2, Z1, dZ1);
    // layer 1
    hipLaunchKernelGGL(k_bwd_weight, dim3(blocks((int64_t)NH * (NI + 1))), dim3(256), 0, st, B, NI, NH, dZ1, X, gW1, gb1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (lr > 0.0f && Madam && Vadam) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
        hipLaunchKernelGGL(k_adam, dim3(blocks(NET_PARAMS)), dim3(256), 0, st, NET_PARAMS, P, G, Madam, Vadam, lr, b1,
                           b2, eps, c1, c2);
    }
    return hipGetLastError();
}
