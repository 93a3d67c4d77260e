// valu_rates.hip -- issue cost of the gfx950 vector instructions the quadrature
// kernel is made of, measured on the device (a standalone executable, not part
// of the library).  Each kernel runs independent dependency chains of one
// instruction kind in registers, 8 waves per SIMD, after a warm-up that brings
// the clocks up; the result is SIMD cycles per wave instruction at the 2.4 GHz
// peak clock.  Prints one JSON object.
//
// Operands differ from lane to lane (as in the quadrature) except in the
// lane-uniform variant, which shows how much of the FMA cost depends on the
// data; the interleaved variant alternates FMAs with and without an SGPR
// operand, as the quadrature's instruction stream does.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int CH = 16;          // independent chains per lane
constexpr int BLOCKS = 4096;    // 256-thread blocks: 16 waves per SIMD on 256 CUs (two rounds of 8)

enum Op { FMAC_V, FMAC_S, MUL_V, ADD_V, SIN_V, RSQ_V, FMA_F64, FMAC_UNIFORM, FMAC_SV, MUL_F64, ADD_F64 };

template <int OP>
__global__ void __launch_bounds__(256) k_rate(float *out, int iters, float s_y)
{
    float lane_term = (float)threadIdx.x;
    if (OP == FMAC_UNIFORM) {   // zero in every lane, but opaque: the operands stay in VGPRs
        lane_term = 0.0f;
        asm volatile("" : "+v"(lane_term));
    }
    const float y = 0.999f + lane_term * 1e-9f;   // a VGPR operand (per-lane unless uniform)
    float acc[CH], x[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        acc[c] = (lane_term + c) * 1e-3f;
        x[c] = 1e-4f * (c + 1) + lane_term * 1e-10f;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (OP == FMAC_V || OP == FMAC_UNIFORM) acc[c] = __builtin_fmaf(x[c], y, acc[c]);
            if (OP == FMAC_SV) acc[c] = __builtin_fmaf(x[c], (c & 1) ? y : s_y, acc[c]);
            if (OP == FMAC_S) acc[c] = __builtin_fmaf(x[c], s_y, acc[c]);   // s_y: an SGPR operand
            if (OP == MUL_V) acc[c] = acc[c] * y;
            if (OP == ADD_V) acc[c] = acc[c] + x[c];
            if (OP == SIN_V) acc[c] = __builtin_amdgcn_sinf(acc[c]);
            if (OP == RSQ_V) acc[c] = __builtin_amdgcn_rsqf(acc[c] + 1.0f);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += acc[c] + x[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int OP>
__global__ void __launch_bounds__(256) k_rate_f64(double *out, int iters)
{
    const double y = 0.999 + threadIdx.x * 1e-12;
    double acc[CH], x[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        acc[c] = (double)(threadIdx.x + c) * 1e-3;
        x[c] = 1e-4 * (c + 1) + threadIdx.x * 1e-13;   // per-lane: a VGPR operand
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (OP == FMA_F64) acc[c] = __builtin_fma(x[c], y, acc[c]);
            if (OP == MUL_F64) acc[c] = acc[c] * y;
            if (OP == ADD_F64) acc[c] = acc[c] + x[c];
        }
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += acc[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int OP>
void launch(float *o, double *od, int iters)
{
    if (OP == FMA_F64 || OP == MUL_F64 || OP == ADD_F64)
        hipLaunchKernelGGL((k_rate_f64<OP>), dim3(BLOCKS), dim3(256), 0, 0, od, iters);
    else hipLaunchKernelGGL((k_rate<OP>), dim3(BLOCKS), dim3(256), 0, 0, o, iters, 0.999f);
}

template <int OP>
double cycles_per_instruction(float *o, double *od, int iters)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
        (void)hipEventRecord(e0);
        launch<OP>(o, od, iters);
        (void)hipEventRecord(e1);
        if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double wave_instr = (double)BLOCKS * 4 * iters * CH;
    return best * 1e-3 * 2.4e9 * 1024.0 / wave_instr;   // SIMD cycles per wave instruction
}

}  // namespace

int main()
{
    float *o = nullptr;
    double *od = nullptr;
    if (hipMalloc(&o, sizeof(float) * BLOCKS * 256) != hipSuccess ||
        hipMalloc(&od, sizeof(double) * BLOCKS * 256) != hipSuccess) {
        fprintf(stderr, "valu_rates: allocation failed\n");
        return 1;
    }
    for (int w = 0; w < 40; ++w) launch<FMAC_V>(o, od, 8192);   // ~0.5 s: clocks up
    if (hipDeviceSynchronize() != hipSuccess) return 2;
    const int it = 8192;
    printf("{\"unit\": \"SIMD cycles per wave64 instruction at 2.4 GHz\", "
           "\"v_fmac_f32 (VGPR operands)\": %.3f, \"v_fmac_f32 (SGPR operand)\": %.3f, \"v_mul_f32\": %.3f, "
           "\"v_add_f32\": %.3f, \"v_sin_f32\": %.3f, \"v_rsq_f32 + v_add_f32\": %.3f, \"v_fma_f64\": %.3f, "
           "\"v_fmac_f32 (lane-uniform data)\": %.3f, \"v_fmac_f32 (SGPR and VGPR operands alternating)\": %.3f, "
           "\"v_mul_f64\": %.3f, \"v_add_f64\": %.3f}\n",
           cycles_per_instruction<FMAC_V>(o, od, it), cycles_per_instruction<FMAC_S>(o, od, it),
           cycles_per_instruction<MUL_V>(o, od, it), cycles_per_instruction<ADD_V>(o, od, it),
           cycles_per_instruction<SIN_V>(o, od, it / 4), cycles_per_instruction<RSQ_V>(o, od, it / 4),
           cycles_per_instruction<FMA_F64>(o, od, it), cycles_per_instruction<FMAC_UNIFORM>(o, od, it),
           cycles_per_instruction<FMAC_SV>(o, od, it), cycles_per_instruction<MUL_F64>(o, od, it),
           cycles_per_instruction<ADD_F64>(o, od, it));
    (void)hipFree(o);
    (void)hipFree(od);
    return 0;
}
