// sc_internal.h -- host-side declarations shared by the C ABI (sc_api.cpp) and
// the kernel translation unit (sc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_quadjob.h"

namespace sc {

// ---- launchers (all asynchronous on `stream`; return hipError_t)
hipError_t launch_node_tables(hipStream_t st, int n_r, int n_phi, double f, const double *r,
                              const double *wr, const double *cphi, const double *sphi, double dphi,
                              double *pos64, float *pos32, double *nrm, double *wgt, double *tan);
// General surface: node records from surface nodes + n dS and boundary nodes + normal + dl.
hipError_t launch_surface_records(hipStream_t st, int n_surf, int n_rim, const double *xyz, const double *ndS,
                                  const double *rim_xyz, const double *rim_n, const double *rim_dl, double *pos64,
                                  float *pos32, double *nrm, double *wgt, double *tan);
// hinv64[q], hinv32[q] = 1 / (2 |r_s|) from the FP64 node records (0 where |r_s| = 0).
hipError_t launch_node_half_inverse(hipStream_t st, int n_tot, const double *pos64, double *hinv64, float *hinv32);
hipError_t launch_obs_prep(hipStream_t st, const double *xyz, int n_obs, int n_obs_pad, double *obs64,
                           float *obs32);
hipError_t launch_tables_from_fields(hipStream_t st, int n_k, int n_surf, int n_tot, const double *k,
                                     const double *pos64, const double *nrm, const double *wgt,
                                     const double *tan, const double *E, const double *B, double *tab64);
// beam: 0 linear Gaussian, 1 radially, 2 azimuthally polarised, 3 Laguerre-Gauss mode set
// (modes: device [n_modes][SC_LG_RECORD] = p, l, ex re, ex im, ey re, ey im, the normalisation
// C_{p,l} (including 1 / w0), unused; unused for the other beams)
constexpr int SC_LG_RECORD = 8;
hipError_t launch_tables_gaussian(hipStream_t st, int n_k, int n_surf, int n_tot, const double *k,
                                  const double *pos64, const double *nrm, const double *wgt,
                                  const double *tan, int beam, double w0, double pol, const double *spectrum,
                                  int consistent, const double *modes, int n_modes, double *tab64);
// FP32 tables from the FP64 ones (tab64), or from FP32 split tables (src32, when tab64 is null)
hipError_t launch_tables_cast(hipStream_t st, int n_k, int n_tot, const double *k, const double *pos64,
                              const double *tab64, const float *src32, float *tab32, int naive);
// Incident power per frequency through the aperture, P[k] = 4 pi sum_surface W Re(E x B^*).(-z):
// from field tables E, B [n_k][n_tot][3] complex, or from the built-in Gaussian beam.
// `part` holds power_partial_count(n_k) doubles of scratch; P is [n_k] (device).
hipError_t launch_power_fields(hipStream_t st, int n_k, int n_surf, int n_tot, const double *nrm, const double *wgt,
                               const double *E, const double *B, double *part, double *P);
hipError_t launch_power_gaussian(hipStream_t st, int n_k, int n_surf, const double *k, const double *pos64,
                                 const double *nrm, const double *wgt, int beam, double w0, double pol,
                                 const double *spectrum, int consistent, const double *modes, int n_modes,
                                 double *part, double *P);
int power_partial_count(int n_k);
// tab[k][node] *= fac[k] (complex128 [n_k]) for the n_cplx complex numbers of each record (4 general,
// 2 factored); exactly one of tab64, tab32 non-null
hipError_t launch_tables_scale(hipStream_t st, int n_k, int n_tot, int n_cplx, const double *fac, double *tab64,
                               float *tab32);
// Factored tables (Jt = u s per node): tabf [n_k][n_tot][4] = (s, rho_t), posf [n_tot][8] =
// (x, y, z, |r_s|, u, 1 / (2|r_s|)) in FP32, tabf64 / posf64 the same in FP64 (each output may be
// NULL);
// *bad (zeroed by the caller) gets bit 0 when some node's current has no single real direction
// within tol32 (relative to its largest |Jt| over k), bit 1 for tol64; bits 2 and 3 when some
// node's charge is not tied to its current (rho_t = -i beta s / k, beta real) within tol32, tol64
// (relative to its largest (|rho_t|^2 + |Jt / k|^2)^1/2).
hipError_t launch_tables_factor(hipStream_t st, int n_k, int n_tot, const double *k, const double *tab64,
                                const float *pos32, const double *pos64, double tol32, double tol64, float *tabf,
                                float *posf, float *betaf, float *tabp, double *tabf64, double *posf64,
                                double *betaf64, unsigned int *bad);
// tabp[r] = (|s|, arg(s) / 2 pi) from the FP32 factored records tabf[r] = (s, rho_t), r < n_rec.
hipError_t launch_tables_polar(hipStream_t st, int64_t n_rec, const float *tabf, float *tabp);
// Maxwell-residual diagnostics (sc_diag.hip).  Stencil results [rows][13 n_pts][3] complex (double
// if is_f64, else float); work holds diag_slots() doubles per (row, point), mx 4 per row, out 1 per
// (row, point).  The time form reads [n_t * 5][13 n_pts][3] (times t_m + (j - 2) dt).
hipError_t launch_maxwell_freq(hipStream_t st, int is_f64, int n_k, int n_pts, double h, const double *k,
                               const void *E, const void *B, double *work, double *mx, double *out);
hipError_t launch_maxwell_time(hipStream_t st, int is_f64, int n_t, int n_pts, double h, double dt, const void *E,
                               const void *B, double *work, double *mx, double *out);
int diag_slots();
// Energy 1/2 dV sum (|2 Re E|^2 + |2 Re B|^2) per time row of [n_t][n_obs][3]; part: energy_partial_count(n_t).
int energy_partial_count(int n_t);
hipError_t launch_energy(hipStream_t st, int is_f64, int n_t, int n_obs, const void *E, const void *B, double half_dv,
                         double *part, double *W);
hipError_t launch_quad(hipStream_t st, int mode, int obs_per_lane, int freq_per_lane, int waves_per_block,
                       int grid, const QuadJob *jobs, int n_jobs, int64_t n_tiles, unsigned int *counter);
hipError_t launch_reduce(hipStream_t st, int mode, const void *partial, int n_chunks, int n_k, int n_obs,
                         int n_obs_pad, const double *k, int b_over_k, void *E, void *B);
hipError_t launch_twiddles(hipStream_t st, int n_k, const double *k, int n_t, const double *t, double dk,
                           double *tw);
hipError_t launch_time(hipStream_t st, int is_f64, int n_k, int n_t, int64_t n_x, const double *tw,
                       const void *F, void *Ft);
hipError_t launch_fill_u32(hipStream_t st, unsigned int *p, unsigned int v, int n);
// *dst = job on the device (the job travels as a kernel argument)
hipError_t launch_store_job(hipStream_t st, const QuadJob &job, QuadJob *dst);

// Occupancy helper: max resident workgroups per CU for a quadrature variant.
int quad_max_blocks_per_cu(int mode, int obs_per_lane, int freq_per_lane, int waves_per_block);

}  // namespace sc
