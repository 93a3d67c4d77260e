// sc_diag.hip -- verification diagnostics of the reflected field (Sec. IV-A):
// Maxwell residuals in the frequency and time domains (eqs. relDiffMaxwellFreq,
// relDiffMaxwellTime) and the electromagnetic energy of the observation set.
//
// The fields come from the hot path evaluated on a finite-difference stencil:
// for point i, stencil row 13 i is the point itself and rows 13 i + 1 + 4 a + j
// (axis a = x, y, z; j = 0..3) sit at offsets -2h, -h, +h, +2h along axis a.
// Derivatives are 4th-order central differences,
//     f' = (f(-2h) - 8 f(-h) + 8 f(h) - f(2h)) / (12 h),
// in space and (time domain) in time.  All arithmetic in FP64.
#include "sc_device.h"
#include "sc_internal.h"

namespace sc {

constexpr int STENCIL = 13;
constexpr int DIAG_SLOTS = 16;   // per (row, point): r1 (3 complex), r2 (3 complex), 4 norms

__device__ __forceinline__ double fd4(double m2, double m1, double p1, double p2, double inv12h)
{
    return ((m2 - p2) + 8.0 * (p1 - m1)) * inv12h;
}

// Real and imaginary parts of component c of stencil row `row` of a [rows][3] complex array.
template <typename T>
__device__ __forceinline__ double cre(const T *F, size_t row, int c) { return (double)F[6 * row + 2 * c]; }
template <typename T>
__device__ __forceinline__ double cim(const T *F, size_t row, int c) { return (double)F[6 * row + 2 * c + 1]; }

// curl of a complex field from its stencil rows (base = first row of the point), part 0 = re, 1 = im
template <typename T>
__device__ __forceinline__ void curl_stencil(const T *F, size_t base, double h, double cr[3], double ci[3])
{
    const double inv = 1.0 / (12.0 * h);
    double Jr[3][3], Ji[3][3];   // J[a][c] = d_a F_c
    for (int a = 0; a < 3; ++a) {
        const size_t r0 = base + 1 + 4 * a;
        for (int c = 0; c < 3; ++c) {
            Jr[a][c] = fd4(cre(F, r0, c), cre(F, r0 + 1, c), cre(F, r0 + 2, c), cre(F, r0 + 3, c), inv);
            Ji[a][c] = fd4(cim(F, r0, c), cim(F, r0 + 1, c), cim(F, r0 + 2, c), cim(F, r0 + 3, c), inv);
        }
    }
    cr[0] = Jr[1][2] - Jr[2][1];
    cr[1] = Jr[2][0] - Jr[0][2];
    cr[2] = Jr[0][1] - Jr[1][0];
    ci[0] = Ji[1][2] - Ji[2][1];
    ci[1] = Ji[2][0] - Ji[0][2];
    ci[2] = Ji[0][1] - Ji[1][0];
}

__device__ __forceinline__ double norm6(const double *re, const double *im)
{
    return sqrt(re[0] * re[0] + re[1] * re[1] + re[2] * re[2] + im[0] * im[0] + im[1] * im[1] + im[2] * im[2]);
}

// Frequency domain, per (k, point):  r1 = curl E - ik B,  r2 = curl B + ik E  and the
// norms |curl E|, |ik B|, |curl B|, |ik E| (at the point itself).
template <typename T>
__global__ void k_maxwell_freq(int n_k, int n_pts, double h, const double *__restrict__ kv,
                               const T *__restrict__ E, const T *__restrict__ B, double *__restrict__ work)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_pts) return;
    const int kk = (int)(idx / n_pts);
    const int i = (int)(idx - (int64_t)kk * n_pts);
    const double k = kv[kk];
    const size_t base = ((size_t)kk * n_pts + i) * STENCIL;
    double eR[3], eI[3], bR[3], bI[3];
    curl_stencil(E, base, h, eR, eI);
    curl_stencil(B, base, h, bR, bI);
    double r1r[3], r1i[3], r2r[3], r2i[3], ikBr[3], ikBi[3], ikEr[3], ikEi[3];
    for (int c = 0; c < 3; ++c) {
        // ik (a + ib) = -k b + i k a
        ikBr[c] = -k * cim(B, base, c);
        ikBi[c] = k * cre(B, base, c);
        ikEr[c] = -k * cim(E, base, c);
        ikEi[c] = k * cre(E, base, c);
        r1r[c] = eR[c] - ikBr[c];
        r1i[c] = eI[c] - ikBi[c];
        r2r[c] = bR[c] + ikEr[c];
        r2i[c] = bI[c] + ikEi[c];
    }
    double *w = work + idx * DIAG_SLOTS;
    for (int c = 0; c < 3; ++c) {
        w[2 * c] = r1r[c];
        w[2 * c + 1] = r1i[c];
        w[6 + 2 * c] = r2r[c];
        w[6 + 2 * c + 1] = r2i[c];
    }
    w[12] = norm6(eR, eI);
    w[13] = norm6(ikBr, ikBi);
    w[14] = norm6(bR, bI);
    w[15] = norm6(ikEr, ikEi);
}

// Time domain, per (t_m, point), with the physical fields 2 Re F:
//   r1 = curl E + dB/dt,  r2 = curl B - dE/dt  and |curl E|, |dB/dt|, |curl B|, |dE/dt|.
// Ft rows: (m * 5 + j) * (13 n_pts) + stencil row, j = 0..4 at t_m + (j - 2) dt.
template <typename T>
__global__ void k_maxwell_time(int n_t, int n_pts, double h, double dt, const T *__restrict__ E,
                               const T *__restrict__ B, double *__restrict__ work)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_t * n_pts) return;
    const int m = (int)(idx / n_pts);
    const int i = (int)(idx - (int64_t)m * n_pts);
    const size_t rows = (size_t)STENCIL * n_pts;
    const size_t pt = (size_t)i * STENCIL;
    const size_t c0 = ((size_t)m * 5 + 2) * rows + pt;   // time t_m, stencil of point i
    double eR[3], eI[3], bR[3], bI[3];
    curl_stencil(E, c0, h, eR, eI);
    curl_stencil(B, c0, h, bR, bI);
    const double inv = 1.0 / (12.0 * dt);
    double dE[3], dB[3], cE[3], cB[3], r1[3], r2[3];
    for (int c = 0; c < 3; ++c) {
        const size_t tm2 = ((size_t)m * 5 + 0) * rows + pt, tm1 = ((size_t)m * 5 + 1) * rows + pt;
        const size_t tp1 = ((size_t)m * 5 + 3) * rows + pt, tp2 = ((size_t)m * 5 + 4) * rows + pt;
        dE[c] = 2.0 * fd4(cre(E, tm2, c), cre(E, tm1, c), cre(E, tp1, c), cre(E, tp2, c), inv);
        dB[c] = 2.0 * fd4(cre(B, tm2, c), cre(B, tm1, c), cre(B, tp1, c), cre(B, tp2, c), inv);
        cE[c] = 2.0 * eR[c];
        cB[c] = 2.0 * bR[c];
        r1[c] = cE[c] + dB[c];
        r2[c] = cB[c] - dE[c];
    }
    const double zero[3] = {0.0, 0.0, 0.0};
    double *w = work + idx * DIAG_SLOTS;
    for (int c = 0; c < 3; ++c) {
        w[2 * c] = r1[c];
        w[2 * c + 1] = 0.0;
        w[6 + 2 * c] = r2[c];
        w[6 + 2 * c + 1] = 0.0;
    }
    w[12] = norm6(cE, zero);
    w[13] = norm6(dB, zero);
    w[14] = norm6(cB, zero);
    w[15] = norm6(dE, zero);
}

// Per row: the maxima of the four norms over the points (max is exact, so the
// result does not depend on the reduction order).
__global__ void __launch_bounds__(256) k_maxwell_max(int n_pts, const double *__restrict__ work,
                                                     double *__restrict__ mx)
{
    __shared__ double red[4][256];
    const int row = blockIdx.x;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n_pts; i += 256) {
        const double *w = work + ((size_t)row * n_pts + i) * DIAG_SLOTS + 12;
        for (int j = 0; j < 4; ++j) m[j] = fmax(m[j], w[j]);
    }
    for (int j = 0; j < 4; ++j) red[j][threadIdx.x] = m[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int j = 0; j < 4; ++j) red[j][threadIdx.x] = fmax(red[j][threadIdx.x], red[j][threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x < 4) mx[(size_t)row * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// |e| = | 2 r1 / (max n1 + max n2) + 2 r2 / (max n3 + max n4) |  per (row, point).
__global__ void k_maxwell_final(int n_rows, int n_pts, const double *__restrict__ work,
                                const double *__restrict__ mx, double *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_rows * n_pts) return;
    const int row = (int)(idx / n_pts);
    const double *M = mx + (size_t)row * 4;
    const double d1 = M[0] + M[1], d2 = M[2] + M[3];
    const double s1 = d1 > 0.0 ? 2.0 / d1 : 0.0, s2 = d2 > 0.0 ? 2.0 / d2 : 0.0;
    const double *w = work + idx * DIAG_SLOTS;
    double acc = 0.0;
    for (int c = 0; c < 6; ++c) {
        const double v = s1 * w[c] + s2 * w[6 + c];
        acc += v * v;
    }
    out[idx] = sqrt(acc);
}

// Energy of the observation set at time row m: 1/2 dV sum_points (|2 Re E|^2 + |2 Re B|^2).
// grid (ENERGY_BLOCKS, n_t); block b sums a fixed point range in a fixed order.
constexpr int ENERGY_BLOCKS = 32;

template <typename T>
__global__ void __launch_bounds__(256) k_energy(int n_obs, const T *__restrict__ E, const T *__restrict__ B,
                                                double *__restrict__ part)
{
    __shared__ double red[256];
    const int m = blockIdx.y;
    const int span = (n_obs + ENERGY_BLOCKS - 1) / ENERGY_BLOCKS;
    const int o0 = blockIdx.x * span, o1 = min(o0 + span, n_obs);
    double acc = 0.0;
    for (int o = o0 + (int)threadIdx.x; o < o1; o += 256) {
        const size_t row = (size_t)m * n_obs + o;
        for (int c = 0; c < 3; ++c) {
            const double e = 2.0 * cre(E, row, c), b = 2.0 * cre(B, row, c);
            acc += e * e + b * b;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)m * ENERGY_BLOCKS + blockIdx.x] = red[0];
}

__global__ void k_energy_finish(int n_t, double half_dv, const double *__restrict__ part, double *__restrict__ W)
{
    const int64_t gm = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gm >= n_t) return;
    const int m = (int)gm;
    double s = 0.0;
    for (int b = 0; b < ENERGY_BLOCKS; ++b) s += part[(size_t)m * ENERGY_BLOCKS + b];
    W[m] = half_dv * s;
}

static inline unsigned int nblk(int64_t n, int bs) { return (unsigned int)((n + bs - 1) / bs); }

hipError_t launch_maxwell_freq(hipStream_t st, int is_f64, int n_k, int n_pts, double h, const double *k,
                               const void *E, const void *B, double *work, double *mx, double *out)
{
    const unsigned int nb = nblk((int64_t)n_k * n_pts, 256);
    if (is_f64)
        hipLaunchKernelGGL((k_maxwell_freq<double>), dim3(nb), dim3(256), 0, st, n_k, n_pts, h, k,
                           (const double *)E, (const double *)B, work);
    else
        hipLaunchKernelGGL((k_maxwell_freq<float>), dim3(nb), dim3(256), 0, st, n_k, n_pts, h, k, (const float *)E,
                           (const float *)B, work);
    hipLaunchKernelGGL(k_maxwell_max, dim3(n_k), dim3(256), 0, st, n_pts, work, mx);
    hipLaunchKernelGGL(k_maxwell_final, dim3(nb), dim3(256), 0, st, n_k, n_pts, work, mx, out);
    return hipGetLastError();
}

hipError_t launch_maxwell_time(hipStream_t st, int is_f64, int n_t, int n_pts, double h, double dt, const void *E,
                               const void *B, double *work, double *mx, double *out)
{
    const unsigned int nb = nblk((int64_t)n_t * n_pts, 256);
    if (is_f64)
        hipLaunchKernelGGL((k_maxwell_time<double>), dim3(nb), dim3(256), 0, st, n_t, n_pts, h, dt,
                           (const double *)E, (const double *)B, work);
    else
        hipLaunchKernelGGL((k_maxwell_time<float>), dim3(nb), dim3(256), 0, st, n_t, n_pts, h, dt, (const float *)E,
                           (const float *)B, work);
    hipLaunchKernelGGL(k_maxwell_max, dim3(n_t), dim3(256), 0, st, n_pts, work, mx);
    hipLaunchKernelGGL(k_maxwell_final, dim3(nb), dim3(256), 0, st, n_t, n_pts, work, mx, out);
    return hipGetLastError();
}

int diag_slots() { return DIAG_SLOTS; }
int energy_partial_count(int n_t) { return ENERGY_BLOCKS * n_t; }

hipError_t launch_energy(hipStream_t st, int is_f64, int n_t, int n_obs, const void *E, const void *B, double half_dv,
                         double *part, double *W)
{
    if (is_f64)
        hipLaunchKernelGGL((k_energy<double>), dim3(ENERGY_BLOCKS, n_t), dim3(256), 0, st, n_obs, (const double *)E,
                           (const double *)B, part);
    else
        hipLaunchKernelGGL((k_energy<float>), dim3(ENERGY_BLOCKS, n_t), dim3(256), 0, st, n_obs, (const float *)E,
                           (const float *)B, part);
    hipLaunchKernelGGL(k_energy_finish, dim3(nblk(n_t, 256)), dim3(256), 0, st, n_t, half_dv, part, W);
    return hipGetLastError();
}

}  // namespace sc
