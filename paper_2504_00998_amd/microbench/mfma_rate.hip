// Sustained matrix-core and vector FMA rates from registers only.
//
// Each wave runs ITER iterations of CH independent accumulator chains of one
// instruction; 256-thread blocks, OCC blocks per CU (256 CUs).  The second of
// two launches is timed with HIP events.  Build and run:
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       -o mfma_rate mfma_rate.hip && ./mfma_rate
//
// These rates bound what the FE step kernels can reach in each precision.
#include <hip/hip_runtime.h>

#include <cstdio>

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <int CH>
__global__ __launch_bounds__(256) void f64_16x16x4(double *out, int iters) {
    double a = threadIdx.x * 1e-3, b = 1.0 + threadIdx.x * 1e-4;
    d4 c[CH];
    for (int i = 0; i < CH; ++i) c[i] = d4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < CH; ++i) c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[i], 0, 0, 0);
    }
    double s = 0;
    for (int i = 0; i < CH; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void f64_4x4x4(double *out, int iters) {
    double a = threadIdx.x * 1e-3, b = 1.0 + threadIdx.x * 1e-4;
    double c[CH];
    for (int i = 0; i < CH; ++i) c[i] = 0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < CH; ++i) c[i] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c[i], 0, 0, 0);
    }
    double s = 0;
    for (int i = 0; i < CH; ++i) s += c[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void f32_16x16x4(float *out, int iters) {
    float a = threadIdx.x * 1e-3f, b = 1.0f + threadIdx.x * 1e-4f;
    f4 c[CH];
    for (int i = 0; i < CH; ++i) c[i] = f4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < CH; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[i], 0, 0, 0);
    }
    float s = 0;
    for (int i = 0; i < CH; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void f64_fma(double *out, int iters) {
    double x[CH];
    for (int i = 0; i < CH; ++i) x[i] = threadIdx.x * 1e-3 + i;
    const double y = 1.0000001;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < CH; ++i) x[i] = __fma_rn(x[i], y, 1e-9);
    double s = 0;
    for (int i = 0; i < CH; ++i) s += x[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <typename K, typename T>
static void run(const char *name, int ch, int occ, K kern, T *buf, int iters, double flops_per_iter_per_wave) {
    const int blocks = 256 * occ;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, 0, buf, iters);
    (void)hipEventRecord(e0);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, 0, buf, iters);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double tf = (double)blocks * 4 * iters * flops_per_iter_per_wave / (ms * 1e-3) / 1e12;
    printf("| %-22s | %2d | %d (%2d) | %8.3f | %6.1f |\n", name, ch, occ, 4 * occ, ms, tf);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

int main() {
    double *d = nullptr;
    float *f = nullptr;
    const int maxb = 256 * 8;
    if (hipMalloc(&d, sizeof(double) * 256 * maxb) != hipSuccess) return 1;
    if (hipMalloc(&f, sizeof(float) * 256 * maxb) != hipSuccess) return 1;
    const int it = 4096;
    printf("| instruction | chains/wave | blocks/CU (waves/CU) | ms | TFLOP/s |\n|---|---|---|---|---|\n");
    for (int occ : {2, 4, 8}) {
        run("v_mfma_f64_16x16x4_f64", 4, occ, f64_16x16x4<4>, d, it, 4 * 2048.0);
        run("v_mfma_f64_4x4x4_4b", 4, occ, f64_4x4x4<4>, d, it, 4 * 512.0);
        run("v_mfma_f64_4x4x4_4b", 8, occ, f64_4x4x4<8>, d, it, 8 * 512.0);
        run("v_mfma_f32_16x16x4_f32", 1, occ, f32_16x16x4<1>, f, it, 1 * 2048.0);
        run("v_mfma_f32_16x16x4_f32", 4, occ, f32_16x16x4<4>, f, it, 4 * 2048.0);
        run("v_fma_f64 (VALU)", 8, occ, f64_fma<8>, d, it, 8 * 64 * 2.0);
        run("v_fma_f64 (VALU)", 16, occ, f64_fma<16>, d, it, 16 * 64 * 2.0);
    }
    (void)hipFree(d);
    (void)hipFree(f);
    return 0;
}
