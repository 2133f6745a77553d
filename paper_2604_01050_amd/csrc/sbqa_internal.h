// Internal declarations shared by the host runtime and the HIP kernels of the
// SBQA library (gfx950). Not part of the public ABI (include/sbqa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace sbqa {

// Contraction path of a context.
enum Path : int32_t { PATH_F32 = 0, PATH_FP8 = 1, PATH_BF16X3 = 2, PATH_CSR = 3 };

// GEMM tiling shared by the dense kernels and the host planner.
// Output tile: GEMM_BM columns c (replicas) x GEMM_BN rows i (spins);
// each k-tile carries GEMM_KB bytes of K per row.
constexpr int GEMM_BM = 128;
constexpr int GEMM_BN = 128;
constexpr int GEMM_KB = 128;
constexpr int GEMM_THREADS = 256;

// Element kinds of the dense GEMM.
enum GemmKind : int32_t { GK_F32 = 0, GK_FP8 = 1, GK_BF16X3 = 2, GK_F64 = 3 };

// Per-step scalars of the fused update (Eqs. 6-7), precomputed on the host in
// float64 and rounded once to float32.
struct StepCoef {
    float kA;        // (a0 - a_n) / R
    float kB;        // c0 / R
    float dt;        // dt
    float kD;        // dt * a0 / R
    float delta_next;  // Delta_{n+1} (Eq. 8) for the operand emitted by this step
};

// Dense GEMM: out[z][Cp][Np] (+= nothing; every tile written once)
//   = A[Cp][Np] (operand f(X), K-contiguous) x B[Np][Np] (J rows, K-contiguous),
// K range of split z: [z*kchunk, (z+1)*kchunk). Cp % GEMM_BM == 0,
// Np % GEMM_BN == 0, kchunk % (GEMM_KB / elem bytes) == 0.
// A2/B2 are the bf16 low parts for GK_BF16X3, ignored otherwise.
// GK_F64 writes double outputs, the others float.
hipError_t launch_gemm(GemmKind kind, const void *A, const void *A2, const void *B,
                       const void *B2, void *out, int Np, int Cp, int splits,
                       hipStream_t st);

// Dense update over state [C][Np] (replica-major): reads Phi partials
// phi[splits][Cp][Np], x_in, y (in place), writes x_out and the next operand
// in the path's format. jp points at J_perp[r][n] with run stride jp_stride.
hipError_t launch_dense_update(Path path, int fmode, int N, int Np, int R, int runs,
                               int Cp, int splits, const float *phi, const float *h,
                               const float *x_in, float *x_out, float *y, void *g,
                               void *g_lo, const float *jp, int64_t jp_stride,
                               StepCoef k, hipStream_t st);

// Operand f(X) for the dense paths from state [C][Np] with threshold delta.
hipError_t launch_dense_operand(Path path, int fmode, int N, int Np, int C, const float *x,
                                void *g, void *g_lo, float delta, hipStream_t st);

// Sum of Phi partials -> phi_out[C][Np] (test hook).
hipError_t launch_sum_partials(int N, int Np, int C, int Cp, int splits, const float *phi,
                               float *out, hipStream_t st);

// CSR fused step over state [N][Cs] (spin-major): gathers of the operand
// (int8 f values, or x itself for ballistic f), pump/ring/kick/drift/wall,
// next operand with delta_next.
hipError_t launch_csr_step(int fmode, int N, int Cs, int R, int runs, const int32_t *row_ptr,
                           const int32_t *col, const float *val, const float *h,
                           const float *x_in, float *x_out, float *y, const int8_t *g_in,
                           int8_t *g_out, const float *jp, int64_t jp_stride, StepCoef k,
                           hipStream_t st);

// Register-resident CSR loop (K steps per cooperative launch); see
// kernels_csr.hip. Arrays are device pointers; NR = resident_rows(N) rows,
// rows N..NR-1 are zero padding.
struct ResidentArgs {
    int N, Cs, R, S, n0, K, fmode, nwg;
    const int32_t *colpad;  // [NR][D] neighbour indices (padding: index 0, weight 0)
    const float *valpad;    // [D][NR] weights, padded with 0
    const float *h;         // [NR]
    float *x, *y;           // [NR][Cs] state, updated in place
    int8_t *g;              // [NR][Cs] operand, updated in place
    const float *jp;        // [runs][S]
    const float *coefA;     // [S]   (a0 - a_n)/R
    const float *delta;     // [S+1] Delta_n
    float kB, dt, kD;
    float *xpub;            // [2][nwg][2][NR] published edge columns
    int *flags;             // [nwg] steps completed (monotonic)
    int *epoch_cnt;         // [nwg] launches started (monotonic)
    int epoch;              // this launch's number (>= 1)
    int *err;               // [1] set on a wait timeout
};
int resident_degree(int maxdeg);        // padded degree D, or -1 when too large
size_t resident_lds_bytes(int N, int D);
int resident_cols();
int resident_rpt(int N);             // rows per thread, or -1 when N is too large
int resident_rows(int N);            // padded row count NR, or -1
int resident_threads();
hipError_t resident_max_blocks(int D, int N, int *blocks_per_cu);
hipError_t launch_csr_resident(const ResidentArgs &a, int D, hipStream_t st);

// CSR operand from state [N][Cs].
hipError_t launch_csr_operand(int fmode, int N, int Cs, int C, const float *x, int8_t *g,
                              float delta, hipStream_t st);

// CSR coupling sum phi[N][Cs] = J f(X) (test hook).
hipError_t launch_csr_fields(int fmode, int N, int Cs, int C, const int32_t *row_ptr,
                             const int32_t *col, const float *val, const float *x,
                             const int8_t *g, float *phi, hipStream_t st);

// Counter-based initial state: x, y ~ U[-amp, amp] from Philox4x32-10 keyed by
// seed, counter (i, c). spin_major selects [N][ld] (CSR) or [C][ld] (dense).
hipError_t launch_init_state(int N, int C, int ld, bool spin_major, uint64_t seed, double amp,
                             float *x, float *y, hipStream_t st);

// Readout spins sign(x) (sign(0) = +1) as float64 +-1 into S[Cp][Np]
// (zero padding) from the state, for the energy GEMM.
hipError_t launch_readout_f64(int N, int Np, int C, int ld, bool spin_major, const float *x,
                              double *S, hipStream_t st);

// int8 spins [count][N] -> float64 S[Cp][Np].
hipError_t launch_spins_to_f64(int N, int Np, int count, const int8_t *spins, double *S,
                               hipStream_t st);

// E[c] = sum_i s_ci (-1/2 sum_z phis[z][c][i] - h_i), fixed-order reduction.
hipError_t launch_energy_reduce(int N, int Np, int count, int Cp, int splits,
                                const double *phis, const double *S, const double *h,
                                double *E, hipStream_t st);

// CSR energies of the readout of x ([N][Cs]) or of given spins.
hipError_t launch_csr_energy_state(int N, int Cs, int C, const int32_t *row_ptr,
                                   const int32_t *col, const double *val, const double *h,
                                   const float *x, double *partial, int nblk_rows, double *E,
                                   hipStream_t st);
hipError_t launch_csr_energy_spins(int N, int count, const int32_t *row_ptr, const int32_t *col,
                                   const double *val, const double *h, const int8_t *spins,
                                   double *E, hipStream_t st);

// Per-run best over replicas with tie -> lowest k; updates best_E/best_step
// when strictly lower and copies the winning readout spins.
hipError_t launch_best_update(int N, int R, int runs, int ld, bool spin_major, const float *x,
                              const double *E, double *best_E, int64_t *best_step,
                              int8_t *best_spins, int64_t step, hipStream_t st);

}  // namespace sbqa
