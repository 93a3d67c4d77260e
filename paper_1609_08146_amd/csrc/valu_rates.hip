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
// operand, as the quadrature's instruction stream does.  The first wave of
// every block also reads the core-cycle counter and the constant-rate wall
// clock around its loop, which gives the clock the SIMDs actually ran at, and
// with it the cycles per instruction at that clock.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int CH = 16;          // independent chains per lane
constexpr int BLOCKS = 4096;    // 256-thread blocks: 16 waves per SIMD on 256 CUs (two rounds of 8)

enum Op { FMAC_V, FMAC_S, MUL_V, ADD_V, SIN_V, RSQ_V, FMA_F64, FMAC_UNIFORM, FMAC_SV, MUL_F64, ADD_F64 };

// clk[2 b], clk[2 b + 1]: core cycles and wall-clock ticks of block b's loop (thread 0)
__device__ __forceinline__ void clock_mark(unsigned long long *clk, bool end)
{
    if (threadIdx.x != 0) return;
    const unsigned long long c = (unsigned long long)clock64(), w = (unsigned long long)wall_clock64();
    if (!end) {
        clk[2 * blockIdx.x] = c;
        clk[2 * blockIdx.x + 1] = w;
    } else {
        clk[2 * blockIdx.x] = c - clk[2 * blockIdx.x];
        clk[2 * blockIdx.x + 1] = w - clk[2 * blockIdx.x + 1];
    }
}

template <int OP>
__global__ void __launch_bounds__(256) k_rate(float *out, unsigned long long *clk, int iters, float s_y)
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
    clock_mark(clk, false);
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
    clock_mark(clk, true);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += acc[c] + x[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int OP>
__global__ void __launch_bounds__(256) k_rate_f64(double *out, unsigned long long *clk, int iters)
{
    const double y = 0.999 + threadIdx.x * 1e-12;
    double acc[CH], x[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        acc[c] = (double)(threadIdx.x + c) * 1e-3;
        x[c] = 1e-4 * (c + 1) + threadIdx.x * 1e-13;   // per-lane: a VGPR operand
    }
    clock_mark(clk, false);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (OP == FMA_F64) acc[c] = __builtin_fma(x[c], y, acc[c]);
            if (OP == MUL_F64) acc[c] = acc[c] * y;
            if (OP == ADD_F64) acc[c] = acc[c] + x[c];
        }
    }
    clock_mark(clk, true);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += acc[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

struct Buffers {
    float *o;
    double *od;
    unsigned long long *clk;   // [2 * BLOCKS]
    double wall_hz;            // wall_clock64 rate
};

template <int OP>
void launch(const Buffers &b, int iters)
{
    if (OP == FMA_F64 || OP == MUL_F64 || OP == ADD_F64)
        hipLaunchKernelGGL((k_rate_f64<OP>), dim3(BLOCKS), dim3(256), 0, 0, b.od, b.clk, iters);
    else hipLaunchKernelGGL((k_rate<OP>), dim3(BLOCKS), dim3(256), 0, 0, b.o, b.clk, iters, 0.999f);
}

struct Rate {
    double cycles;   // SIMD cycles per wave instruction at 2.4 GHz
    double ghz;      // the core clock of the timed launch, from the first wave of each block
};

template <int OP>
Rate measure(const Buffers &b, int iters)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return {-1.0, -1.0};
    float best = 1e30f;
    double ghz = 0.0;
    static unsigned long long h[2 * BLOCKS];
    for (int rep = 0; rep < 4; ++rep) {
        (void)hipEventRecord(e0);
        launch<OP>(b, iters);
        (void)hipEventRecord(e1);
        if (hipEventSynchronize(e1) != hipSuccess) return {-1.0, -1.0};
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && ms < best) {
            best = ms;
            if (hipMemcpy(h, b.clk, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return {-1.0, -1.0};
            double cyc = 0.0, wall = 0.0;
            for (int i = 0; i < BLOCKS; ++i) {
                cyc += (double)h[2 * i];
                wall += (double)h[2 * i + 1];
            }
            ghz = wall > 0.0 ? cyc / wall * b.wall_hz * 1e-9 : -1.0;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double wave_instr = (double)BLOCKS * 4 * iters * CH;
    return {best * 1e-3 * 2.4e9 * 1024.0 / wave_instr, ghz};   // SIMD cycles per wave instruction
}

}  // namespace

int main()
{
    Buffers b{};
    int wall_khz = 0;
    if (hipMalloc(&b.o, sizeof(float) * BLOCKS * 256) != hipSuccess ||
        hipMalloc(&b.od, sizeof(double) * BLOCKS * 256) != hipSuccess ||
        hipMalloc(&b.clk, sizeof(unsigned long long) * 2 * BLOCKS) != hipSuccess ||
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, 0) != hipSuccess || wall_khz <= 0) {
        fprintf(stderr, "valu_rates: set-up failed\n");
        return 1;
    }
    b.wall_hz = 1e3 * wall_khz;
    for (int w = 0; w < 40; ++w) launch<FMAC_V>(b, 8192);   // ~0.5 s: clocks up
    if (hipDeviceSynchronize() != hipSuccess) return 2;
    const int it = 8192;
    const char *names[] = {"v_fmac_f32 (VGPR operands)", "v_fmac_f32 (SGPR operand)", "v_mul_f32", "v_add_f32",
                           "v_sin_f32", "v_rsq_f32 + v_add_f32", "v_fma_f64", "v_fmac_f32 (lane-uniform data)",
                           "v_fmac_f32 (SGPR and VGPR operands alternating)", "v_mul_f64", "v_add_f64"};
    const Rate r[] = {measure<FMAC_V>(b, it), measure<FMAC_S>(b, it), measure<MUL_V>(b, it),
                      measure<ADD_V>(b, it), measure<SIN_V>(b, it / 4), measure<RSQ_V>(b, it / 4),
                      measure<FMA_F64>(b, it), measure<FMAC_UNIFORM>(b, it), measure<FMAC_SV>(b, it),
                      measure<MUL_F64>(b, it), measure<ADD_F64>(b, it)};
    const int n = (int)(sizeof(r) / sizeof(r[0]));
    printf("{\"unit\": \"SIMD cycles per wave64 instruction at 2.4 GHz\"");
    for (int i = 0; i < n; ++i) printf(", \"%s\": %.3f", names[i], r[i].cycles);
    printf(", \"clock_ghz\": {");
    for (int i = 0; i < n; ++i) printf("%s\"%s\": %.3f", i ? ", " : "", names[i], r[i].ghz);
    printf("}, \"cycles_at_measured_clock\": {");
    for (int i = 0; i < n; ++i) printf("%s\"%s\": %.3f", i ? ", " : "", names[i], r[i].cycles * r[i].ghz / 2.4);
    printf("}}\n");
    (void)hipFree(b.o);
    (void)hipFree(b.od);
    (void)hipFree(b.clk);
    return 0;
}
