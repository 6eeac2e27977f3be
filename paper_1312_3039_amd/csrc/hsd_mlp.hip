// Warm-start network: a two-hidden-layer MLP n_in -> h -> h -> n_out with
// ReLU, trained with MSE and Adam, all in FP32 on gfx950.  Its output is a
// starting point for the method (a project extension of the warm start of
// Sect. 4.2).  The dense layers are GEMMs on the matrix cores
// (v_mfma_f32_16x16x4f32); everything else is elementwise or a column sum.
//
// Parameters are packed as W1 (h x n_in), b1 (h), W2 (h x h), b2 (h),
// W3 (n_out x h), b3 (n_out), row-major, y = x W^T + b per layer.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "hsd_host.h"

namespace hsd {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;   // C tile per workgroup (GT x GT)
constexpr int GK = 16;   // K step staged through LDS

// C (M x N, row stride ldc) = op(A) op(B) (+ bias[j]) (ReLU), with
// A(i, k) = A[i*ar + k*ac] and B(k, j) = B[k*br + j*bc] so that transposed
// operands need no copy.  256 threads: four wavefronts, each owning a 32x32
// quarter of the tile as 2x2 MFMA 16x16 blocks; K advances 16 at a time
// through LDS, 4 per MFMA.  MFMA operand layout (16x16x4, one block): lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and holds D[4(l/16)+r][l%16],
// r = 0..3.  Out-of-range elements are loaded as zero and never stored.
template <bool RELU, bool BIAS>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float *__restrict__ A,
                                               int ar, int ac, const float *__restrict__ B, int br,
                                               int bc, float *__restrict__ C, int ldc,
                                               const float *__restrict__ bias) {
    __shared__ float As[GK][GT + 4];
    __shared__ float Bs[GK][GT + 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tm = blockIdx.y * GT, tn = blockIdx.x * GT;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bool a_kfast = (ac == 1);
    const bool b_jfast = (bc == 1);
    for (int k0 = 0; k0 < K; k0 += GK) {
        for (int e = tid; e < GT * GK; e += 256) {
            int i, kk;
            if (a_kfast) { i = e / GK; kk = e % GK; } else { kk = e / GT; i = e % GT; }
            const int gi = tm + i, gk = k0 + kk;
            As[kk][i] = (gi < M && gk < K) ? A[(size_t)gi * ar + (size_t)gk * ac] : 0.f;
        }
        for (int e = tid; e < GT * GK; e += 256) {
            int j, kk;
            if (b_jfast) { kk = e / GT; j = e % GT; } else { j = e / GK; kk = e % GK; }
            const int gj = tn + j, gk = k0 + kk;
            Bs[kk][j] = (gj < N && gk < K) ? B[(size_t)gk * br + (size_t)gj * bc] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK; ks += 4) {
            const int kr = ks + (lane >> 4);
            const float a0 = As[kr][wm + (lane & 15)];
            const float a1 = As[kr][wm + 16 + (lane & 15)];
            const float b0 = Bs[kr][wn + (lane & 15)];
            const float b1 = Bs[kr][wn + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = tm + wm + a * 16 + 4 * (lane >> 4) + r;
                const int j = tn + wn + b * 16 + (lane & 15);
                if (i < M && j < N) {
                    float v = acc[a][b][r];
                    if (BIAS) v += bias[j];
                    if (RELU) v = v > 0.f ? v : 0.f;
                    C[(size_t)i * ldc + j] = v;
                }
            }
}

// dY = 2 (Y - T) / (rows * cols); per-workgroup partial of sum (Y - T)^2.
__global__ void k_mse_grad(const float *Y, const float *T, float *dY, int64_t total, float scale,
                           float *partial) {
    __shared__ float red[MAX_WAVES];
    float s = 0.f;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float d = Y[e] - T[e];
        dY[e] = 2.f * d * scale;
        s += d * d;
    }
    float v[1] = {s};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// loss = sum(partials) * scale (single workgroup, fixed order)
__global__ void k_loss_finish(const float *partial, int np, float scale, float *loss) {
    __shared__ float red[MAX_WAVES];
    float s = 0.f;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
    float v[1] = {s};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) *loss = v[0] * scale;
}

// db[j] = sum_i dY[i][j] (one thread per column, rows in order).
__global__ void k_colsum(const float *dY, int rows, int cols, float *db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += dY[(size_t)i * cols + j];
    db[j] = s;
}

// dH *= (H > 0): backward of ReLU given its output H.
__global__ void k_relu_back(float *dH, const float *H, int64_t total) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
        if (!(H[e] > 0.f)) dH[e] = 0.f;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t total, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

struct MlpLayout {
    size_t total = 0;
    size_t params, grads, m1, m2, H1, H2, Y, dY, dH2, dH1, partial, loss;
    size_t take(size_t bytes) {
        size_t off = total;
        total += (bytes + ALIGN - 1) / ALIGN * ALIGN;
        return off;
    }
};

static int64_t mlp_param_count(int64_t ni, int64_t h, int64_t no) {
    return h * ni + h + h * h + h + no * h + no;
}

static MlpLayout mlp_layout(int ni, int h, int no, int maxb) {
    MlpLayout L;
    const int64_t P = mlp_param_count(ni, h, no);
    L.params = L.take(4 * P);
    L.grads = L.take(4 * P);
    L.m1 = L.take(4 * P);
    L.m2 = L.take(4 * P);
    L.H1 = L.take(4 * (int64_t)maxb * h);
    L.H2 = L.take(4 * (int64_t)maxb * h);
    L.Y = L.take(4 * (int64_t)maxb * no);
    L.dY = L.take(4 * (int64_t)maxb * no);
    L.dH2 = L.take(4 * (int64_t)maxb * h);
    L.dH1 = L.take(4 * (int64_t)maxb * h);
    L.partial = L.take(4 * 1024);
    L.loss = L.take(64);
    return L;
}

}  // namespace hsd

using namespace hsd;

struct hsd_mlp {
    int ni = 0, h = 0, no = 0, maxb = 0;
    int64_t P = 0;
    MlpLayout L;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int64_t step = 0;
    float *ptr(size_t off) const { return reinterpret_cast<float *>(ws + off); }
    // parameter blocks
    float *W1() const { return ptr(L.params); }
    float *b1() const { return W1() + (int64_t)h * ni; }
    float *W2() const { return b1() + h; }
    float *b2() const { return W2() + (int64_t)h * h; }
    float *W3() const { return b2() + h; }
    float *b3() const { return W3() + (int64_t)no * h; }
    float *G(int64_t off) const { return ptr(L.grads) + off; }
};

template <bool RELU, bool BIAS>
static int gemm(hipStream_t s, int M, int N, int K, const float *A, int ar, int ac, const float *B,
                int br, int bc, float *C, int ldc, const float *bias) {
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
    hipLaunchKernelGGL((k_gemm<RELU, BIAS>), grid, dim3(256), 0, s, M, N, K, A, ar, ac, B, br, bc, C,
                       ldc, bias);
    HIP_TRY(hipGetLastError());
    return HSD_OK;
}

extern "C" int hsd_mlp_workspace_bytes(int32_t n_in, int32_t n_hidden, int32_t n_out,
                                       int32_t max_batch, size_t *bytes) {
    if (!bytes || n_in < 1 || n_hidden < 1 || n_out < 1 || max_batch < 1)
        return fail(HSD_ERR_ARG, "bad network dimensions");
    *bytes = mlp_layout(n_in, n_hidden, n_out, max_batch).total;
    return HSD_OK;
}

extern "C" int hsd_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch,
                              void *ws, size_t ws_bytes, void *stream, hsd_mlp_t **out) {
    size_t need = 0;
    int rc = hsd_mlp_workspace_bytes(n_in, n_hidden, n_out, max_batch, &need);
    if (rc) return rc;
    if (!ws || !out) return fail(HSD_ERR_ARG, "null argument");
    if (((uintptr_t)ws) % ALIGN) return fail(HSD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(HSD_ERR_WORKSPACE, "workspace too small");
    hsd_mlp *net = new hsd_mlp();
    net->ni = n_in;
    net->h = n_hidden;
    net->no = n_out;
    net->maxb = max_batch;
    net->P = mlp_param_count(n_in, n_hidden, n_out);
    net->L = mlp_layout(n_in, n_hidden, n_out, max_batch);
    net->ws = (char *)ws;
    net->stream = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(net->P, 256)), dim3(256), 0, net->stream,
                       net->ptr(net->L.m1), net->P, 0.f);
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(net->P, 256)), dim3(256), 0, net->stream,
                       net->ptr(net->L.m2), net->P, 0.f);
    if (hipGetLastError() != hipSuccess) {
        delete net;
        return fail(HSD_ERR_HIP, "fill launch failed");
    }
    *out = net;
    return HSD_OK;
}

extern "C" int64_t hsd_mlp_param_count(const hsd_mlp_t *net) { return net ? net->P : -1; }

extern "C" int hsd_mlp_set_params(hsd_mlp_t *net, const float *params) {
    if (!net || !params) return fail(HSD_ERR_ARG, "null argument");
    HIP_TRY(hipMemcpyAsync(net->W1(), params, 4 * (size_t)net->P, hipMemcpyDeviceToDevice, net->stream));
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(net->P, 256)), dim3(256), 0, net->stream,
                       net->ptr(net->L.m1), net->P, 0.f);
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(net->P, 256)), dim3(256), 0, net->stream,
                       net->ptr(net->L.m2), net->P, 0.f);
    HIP_TRY(hipGetLastError());
    net->step = 0;
    return HSD_OK;
}

extern "C" int hsd_mlp_get_params(hsd_mlp_t *net, float *params) {
    if (!net || !params) return fail(HSD_ERR_ARG, "null argument");
    HIP_TRY(hipMemcpyAsync(params, net->W1(), 4 * (size_t)net->P, hipMemcpyDeviceToDevice, net->stream));
    return HSD_OK;
}

static int mlp_forward_impl(hsd_mlp *net, int B, const float *x, float *y) {
    const int ni = net->ni, h = net->h, no = net->no;
    float *H1 = net->ptr(net->L.H1), *H2 = net->ptr(net->L.H2);
    int rc;
    // H1 = relu(x W1^T + b1): A = x (B x ni), B(k, j) = W1[j][k]
    if ((rc = gemm<true, true>(net->stream, B, h, ni, x, ni, 1, net->W1(), 1, ni, H1, h, net->b1()))) return rc;
    if ((rc = gemm<true, true>(net->stream, B, h, h, H1, h, 1, net->W2(), 1, h, H2, h, net->b2()))) return rc;
    if ((rc = gemm<false, true>(net->stream, B, no, h, H2, h, 1, net->W3(), 1, h, y, no, net->b3()))) return rc;
    return HSD_OK;
}

extern "C" int hsd_mlp_forward(hsd_mlp_t *net, int32_t batch, const float *x, float *y) {
    if (!net || !x || !y) return fail(HSD_ERR_ARG, "null argument");
    if (batch < 1 || batch > net->maxb) return fail(HSD_ERR_ARG, "batch outside [1, max_batch]");
    return mlp_forward_impl(net, batch, x, y);
}

// Gradients of L = mean over all outputs of (y - t)^2 with respect to the
// packed parameters, written to net's gradient buffer; loss to net's loss.
static int mlp_backward_impl(hsd_mlp *net, int B, const float *x, const float *t) {
    const int ni = net->ni, h = net->h, no = net->no;
    hipStream_t s = net->stream;
    float *H1 = net->ptr(net->L.H1), *H2 = net->ptr(net->L.H2);
    float *Y = net->ptr(net->L.Y), *dY = net->ptr(net->L.dY);
    float *dH2 = net->ptr(net->L.dH2), *dH1 = net->ptr(net->L.dH1);
    int rc;
    if ((rc = mlp_forward_impl(net, B, x, Y))) return rc;
    const int64_t tot = (int64_t)B * no;
    const float scale = 1.f / (float)tot;
    const int np = grid_for(tot, 256, 1024);
    hipLaunchKernelGGL(k_mse_grad, dim3(np), dim3(256), 0, s, (const float *)Y, t, dY, tot, scale,
                       net->ptr(net->L.partial));
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, (const float *)net->ptr(net->L.partial), np,
                       scale, net->ptr(net->L.loss));
    HIP_TRY(hipGetLastError());
    const int64_t oW1 = 0, ob1 = oW1 + (int64_t)h * ni, oW2 = ob1 + h, ob2 = oW2 + (int64_t)h * h,
                  oW3 = ob2 + h, ob3 = oW3 + (int64_t)no * h;
    // layer 3: dW3 = dY^T H2 (no x h), db3 = colsum(dY), dH2 = dY W3 (B x h)
    if ((rc = gemm<false, false>(s, no, h, B, dY, 1, no, H2, h, 1, net->G(oW3), h, nullptr))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3((no + 255) / 256), dim3(256), 0, s, (const float *)dY, B, no, net->G(ob3));
    if ((rc = gemm<false, false>(s, B, h, no, dY, no, 1, net->W3(), h, 1, dH2, h, nullptr))) return rc;
    hipLaunchKernelGGL(k_relu_back, dim3(grid_for((int64_t)B * h, 256)), dim3(256), 0, s, dH2,
                       (const float *)H2, (int64_t)B * h);
    // layer 2
    if ((rc = gemm<false, false>(s, h, h, B, dH2, 1, h, H1, h, 1, net->G(oW2), h, nullptr))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3((h + 255) / 256), dim3(256), 0, s, (const float *)dH2, B, h, net->G(ob2));
    if ((rc = gemm<false, false>(s, B, h, h, dH2, h, 1, net->W2(), h, 1, dH1, h, nullptr))) return rc;
    hipLaunchKernelGGL(k_relu_back, dim3(grid_for((int64_t)B * h, 256)), dim3(256), 0, s, dH1,
                       (const float *)H1, (int64_t)B * h);
    // layer 1
    if ((rc = gemm<false, false>(s, h, ni, B, dH1, 1, h, x, ni, 1, net->G(oW1), ni, nullptr))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3((h + 255) / 256), dim3(256), 0, s, (const float *)dH1, B, h, net->G(ob1));
    HIP_TRY(hipGetLastError());
    return HSD_OK;
}

extern "C" int hsd_mlp_gradients(hsd_mlp_t *net, int32_t batch, const float *x, const float *t,
                                 float *grads, float *loss) {
    if (!net || !x || !t) return fail(HSD_ERR_ARG, "null argument");
    if (batch < 1 || batch > net->maxb) return fail(HSD_ERR_ARG, "batch outside [1, max_batch]");
    int rc = mlp_backward_impl(net, batch, x, t);
    if (rc) return rc;
    if (grads)
        HIP_TRY(hipMemcpyAsync(grads, net->ptr(net->L.grads), 4 * (size_t)net->P, hipMemcpyDeviceToDevice,
                               net->stream));
    if (loss) HIP_TRY(hipMemcpyAsync(loss, net->ptr(net->L.loss), 4, hipMemcpyDeviceToDevice, net->stream));
    return HSD_OK;
}

extern "C" int hsd_mlp_train_step(hsd_mlp_t *net, int32_t batch, const float *x, const float *t,
                                  float lr, float *loss) {
    if (!net || !x || !t) return fail(HSD_ERR_ARG, "null argument");
    if (batch < 1 || batch > net->maxb) return fail(HSD_ERR_ARG, "batch outside [1, max_batch]");
    int rc = mlp_backward_impl(net, batch, x, t);
    if (rc) return rc;
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - (float)std::pow(0.9, (double)net->step);
    const float c2 = 1.f - (float)std::pow(0.999, (double)net->step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(net->P, 256)), dim3(256), 0, net->stream, net->W1(),
                       (const float *)net->ptr(net->L.grads), net->ptr(net->L.m1), net->ptr(net->L.m2),
                       net->P, lr, b1, b2, eps, c1, c2);
    HIP_TRY(hipGetLastError());
    if (loss) HIP_TRY(hipMemcpyAsync(loss, net->ptr(net->L.loss), 4, hipMemcpyDeviceToDevice, net->stream));
    return HSD_OK;
}

extern "C" void hsd_mlp_destroy(hsd_mlp_t *net) { delete net; }
