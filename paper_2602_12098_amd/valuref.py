"""Reference stream of plain fp32 FMAs for reading VALU counters: the issue
rate a SIMD sustains on independent v_fmac_f32 instructions (no packed
instructions), against which a kernel's clocks per VALU instruction are
compared.  5 waves per SIMD (5120 one-wave workgroups over 256 CUs), each
20,000 iterations of 24 independent FMA chains, run twice.

Usage: python -m paper_2602_12098_amd.valuref --build DIR   (writes DIR/fma_stream)
then, under rocprofv3 --pmc SQ_INSTS_VALU GRBM_GUI_ACTIVE: DIR/fma_stream
"""
import os
import subprocess
import sys

SOURCE = r"""
#include <hip/hip_runtime.h>
#include <cstdio>
__global__ __launch_bounds__(64) void fma_stream(float *out, int iters) {
    float acc[24];
    for (int c = 0; c < 24; ++c) acc[c] = 0.f;
    float a = 1e-3f * threadIdx.x;
    const float b = 1e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 24; ++c) acc[c] = fmaf(a, b, acc[c]);
        a = __builtin_amdgcn_readfirstlane(__float_as_int(a)) ? a : b;   // keeps the loop from folding
    }
    float s = 0.f;
    for (int c = 0; c < 24; ++c) s += acc[c];
    out[blockIdx.x * 64 + threadIdx.x] = s;
}
int main() {
    const int blocks = 256 * 4 * 5, iters = 20000;
    float *d = nullptr;
    if (hipMalloc(&d, (size_t)blocks * 64 * sizeof(float)) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(e0);
        hipLaunchKernelGGL(fma_stream, dim3(blocks), dim3(64), 0, 0, d, iters);
        hipEventRecord(e1);
        if (hipEventSynchronize(e1) != hipSuccess) return 1;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        const double instr = (double)blocks * iters * 24;   // v_fmac_f32 wave instructions in the loop
        printf("fma_stream: %.3f ms, %.3g FMA wave-instructions, %.1f TFLOP/s\n", ms, instr,
               instr * 64 * 2 / (ms * 1e-3) / 1e12);
    }
    hipFree(d);
    return 0;
}
"""


def build(out_dir: str) -> str:
    os.makedirs(out_dir, exist_ok=True)
    src = os.path.join(out_dir, "fma_stream.hip")
    exe = os.path.join(out_dir, "fma_stream")
    with open(src, "w") as f:
        f.write(SOURCE)
    subprocess.run(["hipcc", "-O3", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-o", exe, src], check=True)
    return exe


if __name__ == "__main__":
    if len(sys.argv) != 3 or sys.argv[1] != "--build":
        raise SystemExit(__doc__)
    print(build(sys.argv[2]))
