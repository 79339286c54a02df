// Warm-start MLP on gfx950: bfloat16 GEMM operands on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), FP32 bias / GELU / MSE /
// Adam, FP32 master weights with a bfloat16 copy for the products.
//
// A project addition on top of the method: the network maps a bond-stretch
// geometry descriptor to UCCSD amplitudes, trained on the converged
// amplitudes that plain VQE produces along the scan (Sec. 3.1 "Results for
// bond stretching" is the scan this stands in for); VQE started from its
// prediction is compared with VQE from the Hartree-Fock point (Eq. 1).
//
// Layer l: z_l = a_{l-1} W_l^T + b_l; a_l = GELU(z_l) (exact erf form) for
// hidden layers; the last layer is linear.  Loss: mean squared error.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.h"

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace vqe {

#define HIPCHK_M(expr)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(VQE_EDEVICE, std::string("HIP error in ") + #expr + ": " +         \
                                         hipGetErrorString(e_));                            \
    } while (0)

// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ __forceinline__ float gelu_f(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ void k_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = f2bf(src[i]);
}

// C[i][j] = sum_k A(i,k) B(k,j) (+ bias[j]);  A(i,k) = A[i*sai + k*sak],
// B(k,j) = B[k*sbk + j*sbj], both bfloat16.  One wave64 per 16x16 tile of C,
// 32 k per matrix instruction.  Operand fragments of
// v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)+r] and
// B[8(l/16)+r][l%16], r = 0..7 (A and B split k the same way, so the sum
// over k does not depend on which k a slot holds); the result
// D[4(l/16)+r][l%16], r = 0..3.
// Epilogue: C (fp32, row stride ldc) = acc + bias; if cbf, cbf[i*ldc + j] =
// bf16(GELU(C)) (act = 1) or bf16(C) (act = 0).
__global__ void __launch_bounds__(64) k_gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A,
                                                  int64_t sai, int64_t sak,
                                                  const uint16_t* __restrict__ B, int64_t sbk,
                                                  int64_t sbj, float* __restrict__ C, int64_t ldc,
                                                  const float* __restrict__ bias,
                                                  uint16_t* __restrict__ cbf, int act) {
    const int lane = threadIdx.x;
    const int ti = blockIdx.y * 16, tj = blockIdx.x * 16;
    const int i = ti + (lane & 15), j = tj + (lane & 15);
    const int kq = (lane >> 4) * 8;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        s16x8 a, b;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int k = k0 + kq + r;
            a[r] = (i < M && k < K) ? short(A[i * sai + k * sak]) : short(0);
            b[r] = (j < N && k < K) ? short(B[k * sbk + j * sbj]) : short(0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       acc, 0, 0, 0);
    }
    const int rq = (lane >> 4) * 4;   // the result rows of this lane
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ii = ti + rq + r, jj = tj + (lane & 15);
        if (ii < M && jj < N) {
            const float c = acc[r] + (bias ? bias[jj] : 0.f);
            C[ii * ldc + jj] = c;
            if (cbf) cbf[ii * ldc + jj] = f2bf(act ? gelu_f(c) : c);
        }
    }
}

// dz = 2 (out - y) / (B N) (fp32 and bf16 copies); loss = mean (out - y)^2,
// summed in a fixed order by one block of kMseThreads threads (each thread's
// strided elements, then a tree); loss_trace[*t] = loss when *t < cap.
constexpr int kMseThreads = 1024;

__global__ void __launch_bounds__(kMseThreads) k_mse(const float* __restrict__ out, const float* __restrict__ y,
                                                     int64_t n, float* __restrict__ dz,
                                                     uint16_t* __restrict__ dzbf, float* __restrict__ loss,
                                                     const int* __restrict__ t, float* __restrict__ trace,
                                                     int cap) {
    __shared__ float red[kMseThreads];
    float acc = 0.f;
    const float sc = 2.0f / float(n);
    for (int64_t k = threadIdx.x; k < n; k += kMseThreads) {
        const float d = out[k] - y[k];
        acc += d * d;
        const float g = sc * d;
        dz[k] = g;
        dzbf[k] = f2bf(g);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kMseThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float l = red[0] / float(n);
        *loss = l;
        if (trace && t && *t < cap) trace[*t] = l;
    }
}

// db[j] = sum_i dz[i][j]: one wave per column j, lane l adding rows l, l + 64,
// ... in order, then the 64 lane sums by a fixed butterfly (lane 0's result).
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ dz, int B, int N,
                                                float* __restrict__ db) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= N) return;   // whole waves
    float s = 0.f;
    for (int i = lane; i < B; i += 64) s += dz[int64_t(i) * N + j];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
    if (lane == 0) db[j] = s;
}

// dz = da * GELU'(z), with a bf16 copy
__global__ void k_gelu_back(const float* __restrict__ da, const float* __restrict__ z, int64_t n,
                            float* __restrict__ dz, uint16_t* __restrict__ dzbf) {
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x) {
        const float g = da[k] * gelu_grad_f(z[k]);
        dz[k] = g;
        dzbf[k] = f2bf(g);
    }
}

// Adam on the fp32 master weights (step count *t is the number of steps
// already taken), then the bf16 copy used by the products.
__global__ void k_adam(int64_t P, float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, uint16_t* __restrict__ pbf,
                       const int* __restrict__ t, float lr, float b1, float b2, float eps) {
    const float step = float(*t + 1);
    const float c1 = 1.0f - powf(b1, step), c2 = 1.0f - powf(b2, step);
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < P;
         k += int64_t(gridDim.x) * blockDim.x) {
        const float gk = g[k];
        const float mk = b1 * m[k] + (1.0f - b1) * gk;
        const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        const float pk = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
        p[k] = pk;
        pbf[k] = f2bf(pk);
    }
}

__global__ void k_tick(int* t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *t += 1;
}

}  // namespace vqe

using namespace vqe;

// ============================================================== C ABI (MLP)

struct vqe_mlp {
    int L = 0;
    std::vector<int> w;             // widths, L + 1
    std::vector<int64_t> woff, boff;  // parameter offsets of W_l and b_l
    int64_t P = 0;
    int dev = 0;
    hipStream_t st = nullptr;
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t* pbf = nullptr;
    int* t = nullptr;               // device step counter
    float* loss = nullptr;
    // batch buffers
    int bcap = 0;
    std::vector<uint16_t*> abf;     // abf[l]: bf16 input of layer l, [B][w[l]]
    std::vector<float*> z;          // z[l]: pre-activation of layer l, [B][w[l+1]]
    float *y = nullptr, *dz = nullptr, *da = nullptr, *x = nullptr;
    uint16_t* dzbf = nullptr;
    float* trace = nullptr;
    int trace_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_batch = 0;
    float graph_hp[4] = {0, 0, 0, 0};
    std::vector<void*> allocs;
    ~vqe_mlp() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(dev);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void* a : allocs) (void)hipFree(a);
        if (st) (void)hipStreamDestroy(st);
        (void)hipSetDevice(cur);
    }
};

namespace {

int mlp_alloc(vqe_mlp* n, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? VQE_ENOMEM : VQE_EDEVICE,
                    std::string("MLP allocation: ") + hipGetErrorString(e));
    n->allocs.push_back(*p);
    return VQE_OK;
}

template <class T>
int mlp_alloc_t(vqe_mlp* n, T** p, size_t count) {
    return mlp_alloc(n, reinterpret_cast<void**>(p), count * sizeof(T));
}

int ensure_batch(vqe_mlp* n, int B) {
    if (B <= n->bcap) return VQE_OK;
    HIPCHK_M(hipStreamSynchronize(n->st));
    // buffers for the new capacity (old ones stay allocated until free)
    int wmax = 0;
    for (int x : n->w) wmax = std::max(wmax, x);
    n->abf.assign(n->L, nullptr);
    n->z.assign(n->L, nullptr);
    for (int l = 0; l < n->L; ++l) {
        if (int rc = mlp_alloc_t(n, &n->abf[l], size_t(B) * n->w[l])) return rc;
        if (int rc = mlp_alloc_t(n, &n->z[l], size_t(B) * n->w[l + 1])) return rc;
    }
    if (int rc = mlp_alloc_t(n, &n->x, size_t(B) * n->w[0])) return rc;
    if (int rc = mlp_alloc_t(n, &n->y, size_t(B) * n->w[n->L])) return rc;
    if (int rc = mlp_alloc_t(n, &n->dz, size_t(B) * wmax)) return rc;
    if (int rc = mlp_alloc_t(n, &n->da, size_t(B) * wmax)) return rc;
    if (int rc = mlp_alloc_t(n, &n->dzbf, size_t(B) * wmax)) return rc;
    n->bcap = B;
    if (n->exec) {
        (void)hipGraphExecDestroy(n->exec);
        n->exec = nullptr;
    }
    if (n->graph) {
        (void)hipGraphDestroy(n->graph);
        n->graph = nullptr;
    }
    return VQE_OK;
}

void gemm(hipStream_t st, int M, int N, int K, const uint16_t* A, int64_t sai, int64_t sak,
          const uint16_t* B, int64_t sbk, int64_t sbj, float* C, int64_t ldc, const float* bias,
          uint16_t* cbf, int act) {
    dim3 grid((N + 15) / 16, (M + 15) / 16);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(64), 0, st, M, N, K, A, sai, sak, B, sbk, sbj, C, ldc,
                       bias, cbf, act);
}

int blocks(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024))); }

// Forward pass for B rows already converted into abf[0].
void enqueue_forward(vqe_mlp* n, int B) {
    for (int l = 0; l < n->L; ++l) {
        const int fi = n->w[l], fo = n->w[l + 1];
        const bool last = l == n->L - 1;
        // z = a W^T + b : A(i,k) = abf[i*fi + k], B(k,j) = W[j*fi + k]
        gemm(n->st, B, fo, fi, n->abf[l], fi, 1, n->pbf + n->woff[l], 1, fi, n->z[l], fo,
             n->p + n->boff[l], last ? nullptr : n->abf[l + 1], last ? 0 : 1);
    }
}

// Loss and gradients (into n->g) for targets n->y; t/trace for the loss record.
void enqueue_backward(vqe_mlp* n, int B, bool record) {
    const int fo_last = n->w[n->L];
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(kMseThreads), 0, n->st, n->z[n->L - 1], n->y,
                       int64_t(B) * fo_last, n->dz, n->dzbf, n->loss, n->t,
                       record ? n->trace : nullptr, n->trace_cap);
    for (int l = n->L - 1; l >= 0; --l) {
        const int fi = n->w[l], fo = n->w[l + 1];
        // dW[j][k] = sum_i dz[i][j] a[i][k]: A(j,i) = dzbf[i*fo + j], B(i,k) = abf[i*fi + k]
        gemm(n->st, fo, fi, B, n->dzbf, 1, fo, n->abf[l], fi, 1, n->g + n->woff[l], fi, nullptr,
             nullptr, 0);
        hipLaunchKernelGGL(k_colsum, dim3((fo + 3) / 4), dim3(256), 0, n->st, n->dz, B, fo,
                           n->g + n->boff[l]);
        if (l > 0) {
            // da[i][k] = sum_j dz[i][j] W[j][k]: A(i,j) = dzbf[i*fo + j], B(j,k) = W[j*fi + k]
            gemm(n->st, B, fi, fo, n->dzbf, fo, 1, n->pbf + n->woff[l], fi, 1, n->da, fi, nullptr,
                 nullptr, 0);
            hipLaunchKernelGGL(k_gelu_back, dim3(blocks(int64_t(B) * fi)), dim3(256), 0, n->st,
                               n->da, n->z[l - 1], int64_t(B) * fi, n->dz, n->dzbf);
        }
    }
}

int check_rows(const vqe_mlp* n, int B, const float* x) {
    if (!n || !x) return fail(VQE_EINVAL, "null pointer argument");
    if (B < 1 || B > 65536) return fail(VQE_ERANGE, "batch must be in [1, 65536]");
    if (!std::all_of(x, x + int64_t(B) * n->w[0], [](float v) { return std::isfinite(v); }))
        return fail(VQE_EINVAL, "non-finite input");
    return VQE_OK;
}

}  // namespace

extern "C" int vqe_mlp_create(int n_layers, const int32_t* widths, void* stream, vqe_mlp** out) {
    if (!out || !widths) return fail(VQE_EINVAL, "null pointer argument");
    *out = nullptr;
    if (n_layers < 1 || n_layers > 8) return fail(VQE_ERANGE, "n_layers must be in [1, 8]");
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1 || widths[l] > 8192) return fail(VQE_ERANGE, "widths must be in [1, 8192]");
    auto* n = new vqe_mlp();
    std::unique_ptr<vqe_mlp> guard(n);
    n->L = n_layers;
    n->w.assign(widths, widths + n_layers + 1);
    for (int l = 0; l < n_layers; ++l) {
        n->woff.push_back(n->P);
        n->P += int64_t(n->w[l]) * n->w[l + 1];
        n->boff.push_back(n->P);
        n->P += n->w[l + 1];
    }
    (void)stream;   // the network orders its work on a stream of its own
    HIPCHK_M(hipGetDevice(&n->dev));
    HIPCHK_M(hipStreamCreateWithFlags(&n->st, hipStreamNonBlocking));
    if (int rc = mlp_alloc_t(n, &n->p, n->P)) return rc;
    if (int rc = mlp_alloc_t(n, &n->m, n->P)) return rc;
    if (int rc = mlp_alloc_t(n, &n->v, n->P)) return rc;
    if (int rc = mlp_alloc_t(n, &n->g, n->P)) return rc;
    if (int rc = mlp_alloc_t(n, &n->pbf, n->P)) return rc;
    if (int rc = mlp_alloc_t(n, &n->t, 1)) return rc;
    if (int rc = mlp_alloc_t(n, &n->loss, 1)) return rc;
    HIPCHK_M(hipMemsetAsync(n->p, 0, n->P * sizeof(float), n->st));
    HIPCHK_M(hipMemsetAsync(n->pbf, 0, n->P * sizeof(uint16_t), n->st));
    HIPCHK_M(hipMemsetAsync(n->m, 0, n->P * sizeof(float), n->st));
    HIPCHK_M(hipMemsetAsync(n->v, 0, n->P * sizeof(float), n->st));
    HIPCHK_M(hipMemsetAsync(n->t, 0, sizeof(int), n->st));
    HIPCHK_M(hipStreamSynchronize(n->st));
    *out = guard.release();
    return VQE_OK;
}

extern "C" int vqe_mlp_n_params(const vqe_mlp* n, int64_t* count) {
    if (!n || !count) return fail(VQE_EINVAL, "null pointer argument");
    *count = n->P;
    return VQE_OK;
}

extern "C" int vqe_mlp_set_params(vqe_mlp* n, const float* params) {
    if (!n || !params) return fail(VQE_EINVAL, "null pointer argument");
    if (!std::all_of(params, params + n->P, [](float v) { return std::isfinite(v); }))
        return fail(VQE_EINVAL, "non-finite parameter");
    HIPCHK_M(hipMemcpyAsync(n->p, params, n->P * sizeof(float), hipMemcpyHostToDevice, n->st));
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n->P)), dim3(256), 0, n->st, n->p, n->pbf, n->P);
    HIPCHK_M(hipMemsetAsync(n->m, 0, n->P * sizeof(float), n->st));
    HIPCHK_M(hipMemsetAsync(n->v, 0, n->P * sizeof(float), n->st));
    HIPCHK_M(hipMemsetAsync(n->t, 0, sizeof(int), n->st));
    HIPCHK_M(hipGetLastError());
    HIPCHK_M(hipStreamSynchronize(n->st));
    return VQE_OK;
}

extern "C" int vqe_mlp_get_params(const vqe_mlp* n, float* params) {
    if (!n || !params) return fail(VQE_EINVAL, "null pointer argument");
    HIPCHK_M(hipMemcpyAsync(params, n->p, n->P * sizeof(float), hipMemcpyDeviceToHost, n->st));
    HIPCHK_M(hipStreamSynchronize(n->st));
    return VQE_OK;
}

extern "C" int vqe_mlp_forward(vqe_mlp* n, int B, const float* x, float* y) {
    if (int rc = check_rows(n, B, x)) return rc;
    if (!y) return fail(VQE_EINVAL, "null output");
    if (int rc = ensure_batch(n, B)) return rc;
    HIPCHK_M(hipMemcpyAsync(n->x, x, size_t(B) * n->w[0] * sizeof(float), hipMemcpyHostToDevice,
                            n->st));
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(int64_t(B) * n->w[0])), dim3(256), 0, n->st, n->x,
                       n->abf[0], int64_t(B) * n->w[0]);
    enqueue_forward(n, B);
    HIPCHK_M(hipGetLastError());
    HIPCHK_M(hipMemcpyAsync(y, n->z[n->L - 1], size_t(B) * n->w[n->L] * sizeof(float),
                            hipMemcpyDeviceToHost, n->st));
    HIPCHK_M(hipStreamSynchronize(n->st));
    return VQE_OK;
}

extern "C" int vqe_mlp_loss_grad(vqe_mlp* n, int B, const float* x, const float* y, float* loss,
                                 float* grad) {
    if (int rc = check_rows(n, B, x)) return rc;
    if (!y || !loss) return fail(VQE_EINVAL, "null pointer argument");
    if (int rc = ensure_batch(n, B)) return rc;
    HIPCHK_M(hipMemcpyAsync(n->x, x, size_t(B) * n->w[0] * sizeof(float), hipMemcpyHostToDevice,
                            n->st));
    HIPCHK_M(hipMemcpyAsync(n->y, y, size_t(B) * n->w[n->L] * sizeof(float), hipMemcpyHostToDevice,
                            n->st));
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(int64_t(B) * n->w[0])), dim3(256), 0, n->st, n->x,
                       n->abf[0], int64_t(B) * n->w[0]);
    enqueue_forward(n, B);
    enqueue_backward(n, B, false);
    HIPCHK_M(hipGetLastError());
    HIPCHK_M(hipMemcpyAsync(loss, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->st));
    if (grad)
        HIPCHK_M(hipMemcpyAsync(grad, n->g, n->P * sizeof(float), hipMemcpyDeviceToHost, n->st));
    HIPCHK_M(hipStreamSynchronize(n->st));
    return VQE_OK;
}

extern "C" int vqe_mlp_train(vqe_mlp* n, int B, const float* x, const float* y, int steps, float lr,
                             float beta1, float beta2, float eps, float* loss_trace) {
    if (int rc = check_rows(n, B, x)) return rc;
    if (!y) return fail(VQE_EINVAL, "null targets");
    if (steps < 0) return fail(VQE_ERANGE, "steps < 0");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(VQE_EINVAL, "invalid Adam hyper-parameters");
    if (!std::all_of(y, y + int64_t(B) * n->w[n->L], [](float v) { return std::isfinite(v); }))
        return fail(VQE_EINVAL, "non-finite target");
    if (int rc = ensure_batch(n, B)) return rc;
    // loss trace indexed by the step counter relative to this call
    int t0 = 0;
    HIPCHK_M(hipMemcpyAsync(&t0, n->t, sizeof(int), hipMemcpyDeviceToHost, n->st));
    HIPCHK_M(hipStreamSynchronize(n->st));
    if (n->trace_cap < t0 + steps) {
        void* tr = nullptr;
        if (int rc = mlp_alloc(n, &tr, size_t(t0 + steps + 1024) * sizeof(float))) return rc;
        n->trace = static_cast<float*>(tr);
        n->trace_cap = t0 + steps + 1024;
        if (n->exec) {   // the captured graph refers to the old trace buffer
            (void)hipGraphExecDestroy(n->exec);
            n->exec = nullptr;
            (void)hipGraphDestroy(n->graph);
            n->graph = nullptr;
        }
    }
    HIPCHK_M(hipMemcpyAsync(n->x, x, size_t(B) * n->w[0] * sizeof(float), hipMemcpyHostToDevice,
                            n->st));
    HIPCHK_M(hipMemcpyAsync(n->y, y, size_t(B) * n->w[n->L] * sizeof(float), hipMemcpyHostToDevice,
                            n->st));
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(int64_t(B) * n->w[0])), dim3(256), 0, n->st, n->x,
                       n->abf[0], int64_t(B) * n->w[0]);
    const float hp[4] = {lr, beta1, beta2, eps};
    if (n->exec && (n->graph_batch != B || std::memcmp(hp, n->graph_hp, sizeof(hp)) != 0)) {
        (void)hipGraphExecDestroy(n->exec);
        n->exec = nullptr;
        (void)hipGraphDestroy(n->graph);
        n->graph = nullptr;
    }
    if (!n->exec) {
        // one training step: forward, loss + backward, Adam, step counter
        HIPCHK_M(hipStreamBeginCapture(n->st, hipStreamCaptureModeThreadLocal));
        enqueue_forward(n, B);
        enqueue_backward(n, B, true);
        hipLaunchKernelGGL(k_adam, dim3(blocks(n->P)), dim3(256), 0, n->st, n->P, n->p, n->m, n->v,
                           n->g, n->pbf, n->t, lr, beta1, beta2, eps);
        hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, n->st, n->t);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(n->st, &g);
        n->graph = g;
        HIPCHK_M(ce);
        HIPCHK_M(hipGraphInstantiate(&n->exec, n->graph, nullptr, nullptr, 0));
        n->graph_batch = B;
        std::memcpy(n->graph_hp, hp, sizeof(hp));
    }
    for (int s = 0; s < steps; ++s) HIPCHK_M(hipGraphLaunch(n->exec, n->st));
    if (loss_trace && steps > 0)
        HIPCHK_M(hipMemcpyAsync(loss_trace, n->trace + t0, size_t(steps) * sizeof(float),
                                hipMemcpyDeviceToHost, n->st));
    HIPCHK_M(hipStreamSynchronize(n->st));
    return VQE_OK;
}

extern "C" void vqe_mlp_free(vqe_mlp* n) { delete n; }
