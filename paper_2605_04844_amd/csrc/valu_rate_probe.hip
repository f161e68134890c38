// VALU issue-rate probe (not part of libquadbox): eight independent
// non-packed FP32 FMA chains per lane (then MUL chains, then exp), 2048
// workgroups of 256 lanes so that every SIMD holds 8 waves, timed with HIP
// events; prints lane-instructions per second.  Measures the sustained rate
// of plain single-issue VALU work that the render's roofline is read against.
// Build and run on the GPU (from the repository root):
//   hipcc --offload-arch=gfx950 -O3 -ffp-contract=off -Xclang -target-feature \
//         -Xclang -packed-fp32-ops -o valu_rate paper_2605_04844_amd/csrc/valu_rate_probe.hip
//   ./valu_rate 100000
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(float* out, int iters, float a, float b)
{
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (float)(threadIdx.x + j) * 1e-6f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (MODE == 0) x[j] = fmaf(x[j], a, b);
            else if (MODE == 1) x[j] = x[j] * a;
            else x[j] = __expf(x[j] * a) * b;
        }
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main(int argc, char** argv)
{
    int grid = 2048, block = 256, iters = argc > 1 ? atoi(argv[1]) : 20000;
    float* out;
    if (hipMalloc(&out, sizeof(float) * grid * block) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    const char* names[3] = {"fma", "mul", "exp+mul"};
    for (int mode = 0; mode < 3; ++mode) {
        for (int rep = 0; rep < 3; ++rep) {
            if (hipEventRecord(e0, 0) != hipSuccess) return 2;
            if (mode == 0) hipLaunchKernelGGL(k_probe<0>, dim3(grid), dim3(block), 0, 0, out, iters, 0.9999f, 1e-7f);
            else if (mode == 1) hipLaunchKernelGGL(k_probe<1>, dim3(grid), dim3(block), 0, 0, out, iters, 0.9999f, 1e-7f);
            else hipLaunchKernelGGL(k_probe<2>, dim3(grid), dim3(block), 0, 0, out, iters, -0.5f, 0.5f);
            if (hipEventRecord(e1, 0) != hipSuccess) return 2;
            if (hipEventSynchronize(e1) != hipSuccess) return 2;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 2;
            double lane_ops = (double)grid * block * iters * 8.0 * (mode == 2 ? 2.0 : 1.0);
            printf("%s rep %d: %.3f ms, %.2f T lane-instructions/s\n", names[mode], rep, ms, lane_ops / (ms * 1e-3) / 1e12);
        }
    }
    return hipFree(out) == hipSuccess ? 0 : 3;
}
