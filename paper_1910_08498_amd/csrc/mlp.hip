// Learned configuration predictor: a small multilayer perceptron trained on
// the autotuner's own timings (features of a workload -> scores over the
// tuning space).  The paper points to learning from tuning data as related
// and future work (Sect. 2; Sect. 6); these kernels run its training and
// inference on the GPU.
//
// Parameters live in one float buffer, row-major [in][out] weights then
// biases: W1[n_in][H], b1[H], W2[H][H], b2[H], W3[H][C], b3[C].
// Activations of a mini-batch of B rows live in a caller workspace:
// a1[B][H], a2[B][H], p[B][C] (pre-activations a1, a2; probabilities p),
// then gradient scratch dz[B][C], d2[B][H], d1[B][H] and the gradient
// vector (same layout as the parameters).
//
// The layers are tiny (H = 64, C ~ 130, B <= a few hundred), so each kernel
// maps one thread to one output element and loops over the reduction
// dimension; matrix cores would not pay at these sizes.
#include <hip/hip_runtime.h>

namespace recon {

namespace {

// out[b][j] = sum_k act(in[b][k]) W[k][j] + bias[j]; act = relu when relu_in.
__global__ void k_dense(const float *__restrict__ in, int K, bool relu_in, const float *__restrict__ Wt,
                        const float *__restrict__ bias, float *__restrict__ out, int B, int J)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * J) return;
    const int b = idx / J, j = idx - b * J;
    float acc = bias[j];
    for (int k = 0; k < K; ++k) {
        float v = in[b * K + k];
        if (relu_in) v = fmaxf(v, 0.f);
        acc = fmaf(v, Wt[k * J + j], acc);
    }
    out[idx] = acc;
}

// Row softmax in place (one thread per row); optional loss and dz = (p - y) / B.
__global__ void k_softmax_xent(float *__restrict__ zp, const float *__restrict__ y, float *__restrict__ dz,
                               float *__restrict__ row_loss, int B, int C)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float *z = zp + b * C;
    float m = z[0];
    for (int c = 1; c < C; ++c) m = fmaxf(m, z[c]);
    float s = 0.f;
    for (int c = 0; c < C; ++c) s += expf(z[c] - m);
    const float logs = logf(s);
    float l = 0.f;
    for (int c = 0; c < C; ++c) {
        const float lp = z[c] - m - logs;
        const float p = expf(lp);
        z[c] = p;
        if (y) {
            const float yc = y[b * C + c];
            l -= yc * lp;
            dz[b * C + c] = (p - yc) / static_cast<float>(B);
        }
    }
    if (row_loss) row_loss[b] = l;
}

// Weight gradient gW[k][j] = sum_b act(in[b][k]) d[b][j]; bias gradient
// gb[j] = sum_b d[b][j] (computed by the threads of row k = K).
__global__ void k_dense_grad(const float *__restrict__ in, int K, bool relu_in, const float *__restrict__ d,
                             float *__restrict__ gW, float *__restrict__ gb, int B, int J)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (K + 1) * J) return;
    const int k = idx / J, j = idx - k * J;
    float acc = 0.f;
    if (k < K) {
        for (int b = 0; b < B; ++b) {
            float v = in[b * K + k];
            if (relu_in) v = fmaxf(v, 0.f);
            acc = fmaf(v, d[b * J + j], acc);
        }
        gW[k * J + j] = acc;
    } else {
        for (int b = 0; b < B; ++b) acc += d[b * J + j];
        gb[j] = acc;
    }
}

// Back through a layer: dprev[b][k] = (sum_j d[b][j] W[k][j]) * relu'(a[b][k]).
__global__ void k_dense_back(const float *__restrict__ d, const float *__restrict__ Wt, const float *__restrict__ a,
                             float *__restrict__ dprev, int B, int K, int J)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * K) return;
    const int b = idx / K, k = idx - b * K;
    float acc = 0.f;
    for (int j = 0; j < J; ++j) acc = fmaf(d[b * J + j], Wt[k * J + j], acc);
    dprev[idx] = a[idx] > 0.f ? acc : 0.f;
}

__global__ void k_sgd(float *__restrict__ p, const float *__restrict__ g, float lr, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = fmaf(-lr, g[i], p[i]);
}

__global__ void k_sum(const float *__restrict__ v, int n, float *__restrict__ out)
{
    // single-wave reduction; n is a mini-batch size
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if (threadIdx.x == 0) *out = s / static_cast<float>(n);
}

inline unsigned blocks_for(long n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

size_t mlp_param_count(int n_in, int H, int C)
{
    return static_cast<size_t>(n_in) * H + H + static_cast<size_t>(H) * H + H + static_cast<size_t>(H) * C + C;
}

size_t mlp_ws_floats(int n_in, int H, int C, int B)
{
    // a1, a2, p, dz, d2, d1, row loss, gradients
    return static_cast<size_t>(B) * (2 * H + C) + static_cast<size_t>(B) * (C + 2 * H) + B +
           mlp_param_count(n_in, H, C);
}

// Inference: probabilities [B][C] into `probs` (caller buffer).
hipError_t mlp_forward(const float *params, int n_in, int H, int C, const float *x, int B, float *ws, float *probs,
                       hipStream_t st)
{
    float *a1 = ws, *a2 = a1 + static_cast<size_t>(B) * H, *p = probs;
    const int ob1 = n_in * H, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + H * C;
    hipLaunchKernelGGL(k_dense, dim3(blocks_for(static_cast<long>(B) * H)), dim3(256), 0, st, x, n_in, false, params,
                       params + ob1, a1, B, H);
    hipLaunchKernelGGL(k_dense, dim3(blocks_for(static_cast<long>(B) * H)), dim3(256), 0, st, a1, H, true,
                       params + oW2, params + ob2, a2, B, H);
    hipLaunchKernelGGL(k_dense, dim3(blocks_for(static_cast<long>(B) * C)), dim3(256), 0, st, a2, H, true,
                       params + oW3, params + ob3, p, B, C);
    hipLaunchKernelGGL(k_softmax_xent, dim3(blocks_for(B)), dim3(256), 0, st, p, nullptr, nullptr, nullptr, B, C);
    return hipGetLastError();
}

// One step of gradient descent on the mean cross-entropy of a mini-batch:
// forward, softmax cross-entropy, backward, and params -= lr * grad.  The
// gradient is left in `grads_out` when given (else in the workspace) and the
// batch loss in `loss` when given.
hipError_t mlp_train_step(float *params, int n_in, int H, int C, const float *x, const float *y, int B, float lr,
                          float *ws, float *loss, float *grads_out, hipStream_t st)
{
    float *a1 = ws, *a2 = a1 + static_cast<size_t>(B) * H, *p = a2 + static_cast<size_t>(B) * H;
    float *dz = p + static_cast<size_t>(B) * C, *d2 = dz + static_cast<size_t>(B) * C;
    float *d1 = d2 + static_cast<size_t>(B) * H, *rl = d1 + static_cast<size_t>(B) * H;
    float *g = grads_out ? grads_out : rl + B;
    const int ob1 = n_in * H, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + H * C;
    const int np = static_cast<int>(mlp_param_count(n_in, H, C));
    // forward
    hipLaunchKernelGGL(k_dense, dim3(blocks_for(static_cast<long>(B) * H)), dim3(256), 0, st, x, n_in, false, params,
                       params + ob1, a1, B, H);
    hipLaunchKernelGGL(k_dense, dim3(blocks_for(static_cast<long>(B) * H)), dim3(256), 0, st, a1, H, true,
                       params + oW2, params + ob2, a2, B, H);
    hipLaunchKernelGGL(k_dense, dim3(blocks_for(static_cast<long>(B) * C)), dim3(256), 0, st, a2, H, true,
                       params + oW3, params + ob3, p, B, C);
    hipLaunchKernelGGL(k_softmax_xent, dim3(blocks_for(B)), dim3(256), 0, st, p, y, dz, rl, B, C);
    // backward
    hipLaunchKernelGGL(k_dense_grad, dim3(blocks_for(static_cast<long>(H + 1) * C)), dim3(256), 0, st, a2, H, true,
                       dz, g + oW3, g + ob3, B, C);
    hipLaunchKernelGGL(k_dense_back, dim3(blocks_for(static_cast<long>(B) * H)), dim3(256), 0, st, dz, params + oW3,
                       a2, d2, B, H, C);
    hipLaunchKernelGGL(k_dense_grad, dim3(blocks_for(static_cast<long>(H + 1) * H)), dim3(256), 0, st, a1, H, true,
                       d2, g + oW2, g + ob2, B, H);
    hipLaunchKernelGGL(k_dense_back, dim3(blocks_for(static_cast<long>(B) * H)), dim3(256), 0, st, d2, params + oW2,
                       a1, d1, B, H, H);
    hipLaunchKernelGGL(k_dense_grad, dim3(blocks_for(static_cast<long>(n_in + 1) * H)), dim3(256), 0, st, x, n_in,
                       false, d1, g, g + ob1, B, H);
    if (loss) hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, st, rl, B, loss);
    if (lr != 0.f) hipLaunchKernelGGL(k_sgd, dim3(blocks_for(np)), dim3(256), 0, st, params, g, lr, np);
    return hipGetLastError();
}

}  // namespace recon
