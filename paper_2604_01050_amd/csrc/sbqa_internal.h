// Internal declarations shared by the host runtime and the HIP kernels of the
// SBQA library (gfx950). Not part of the public ABI (include/sbqa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace sbqa {

// Contraction path of a context.
// PATH_FP8PK / PATH_FP4PK: the fp8 / fp4 contraction with J = +-1 stored as
// one bit per coupling.
enum Path : int32_t {
    PATH_F32 = 0, PATH_FP8 = 1, PATH_BF16X3 = 2, PATH_CSR = 3, PATH_I8 = 4, PATH_FP8PK = 5,
    PATH_FP4 = 6, PATH_FP4PK = 7
};
constexpr bool path_fp4(Path p) { return p == PATH_FP4 || p == PATH_FP4PK; }
constexpr bool path_packed(Path p) { return p == PATH_FP8PK || p == PATH_FP4PK; }

// Tiling of the fp64 energy GEMM (row-major operands).
// Output tile: GEMM_BM columns c (replicas) x GEMM_BN rows i (spins);
// each k-tile carries GEMM_KB bytes of K per row.
constexpr int GEMM_BM = 128;
constexpr int GEMM_BN = 128;
constexpr int GEMM_KB = 128;
constexpr int GEMM_THREADS = 256;

// Order of a state buffer (x, y, and the CSR operand) in device memory:
//   ORDER_SPIN_MAJOR    [rows][ld]: CSR contexts stepped one launch per step;
//   ORDER_REPLICA_MAJOR [C][ld]:    dense contexts;
//   ORDER_COLBLOCK8     [C/8][ld][8] (ld = padded rows): CSR contexts of the
//                       register-resident loop, whose workgroups own 8
//                       consecutive replica columns for every spin, so that a
//                       workgroup's state is one contiguous run.
enum StateOrder : int32_t { ORDER_SPIN_MAJOR = 0, ORDER_REPLICA_MAJOR = 1, ORDER_COLBLOCK8 = 2 };
__host__ __device__ inline int64_t state_off(int order, int ld, int i, int c) {
    return order == ORDER_SPIN_MAJOR      ? (int64_t)i * ld + c
           : order == ORDER_REPLICA_MAJOR ? (int64_t)c * ld + i
                                          : ((int64_t)(c >> 3) * ld + i) * 8 + (c & 7);
}

// Per-step scalars of the fused update (Eqs. 6-7), precomputed on the host in
// float64 and rounded once to float32.
struct StepCoef {
    float kA;        // (a0 - a_n) / R
    float kB;        // c0 / R
    float dt;        // dt
    float kD;        // dt * a0 / R
    float delta_next;  // Delta_{n+1} (Eq. 8) for the operand emitted by this step
};

// fp64 GEMM for energies: out[z][Cp][Np] = A[Cp][Np] x B[Np][Np] over the K
// range of split z (both operands row-major, K-contiguous). Cp % GEMM_BM == 0,
// Np % GEMM_BN == 0, Np*8 % (splits*GEMM_KB) == 0.
hipError_t launch_gemm_f64(const double *A, const double *B, double *out, int Np, int Cp, int splits,
                           hipStream_t st);

// ---- dense contraction path -------------------------------------------------
// The coupling matrix J and the operand f(X) of the dense paths are stored as
// 2 KiB fragments ("fragment-tiled"): fragment (rb, kc) holds rows
// 16rb..16rb+15 and K bytes [128kc, 128kc+128); inside it, byte
// h*1024 + l*16 + e holds row 16rb + l%16, K byte 32*(l/16) + 16h + e.
// Lane l of a wave loads bytes l*16 and 1024 + l*16 of a fragment: exactly
// the 32 K bytes it feeds to a 16x16 MFMA. Row blocks are grouped G at a
// time (G = DENSE_TN/16 for J, mbw for the operand); a group is one
// contiguous run, ordered by kc and then by row block, so the fragments a
// workgroup (J) or a wave (operand) needs for one K chunk are adjacent and a
// group's whole K range streams sequentially.
constexpr int FRAG_BYTES = 2048;
constexpr int DENSE_TN = 64;        // J rows (spins) per workgroup: 4 row blocks
constexpr int DENSE_THREADS = 256;  // 4 waves

// Element bytes of the contraction operands (fp4: two elements per byte,
// reported as 1 with path_kpc carrying the difference).
constexpr int path_ebytes(Path p) { return p == PATH_F32 ? 4 : p == PATH_BF16X3 ? 2 : 1; }
// K elements per 128-byte fragment row (one K chunk).
constexpr int path_kpc(Path p) { return path_fp4(p) ? 256 : 128 / path_ebytes(p); }
// K chunks of a row of Np elements.
constexpr int dense_nkc(Path p, int Np) { return Np / path_kpc(p); }
// Bit-packed J: a 16 x kpc fragment in 256 (fp8) or 512 (fp4) bytes, one or
// two dwords per lane.
constexpr int pk_frag_bytes(Path p) { return path_kpc(p) * 2; }
// Device bytes of one plane of a [rows][Np] fragment-tiled matrix.
inline int64_t dense_plane_bytes(Path p, int64_t rows, int Np) { return rows * (int64_t)dense_nkc(p, Np) * 128; }
// Device bytes of the contraction copy of J (one plane).
inline int64_t dense_j_bytes(Path p, int Np) {
    return path_packed(p) ? (int64_t)Np * Np / 8 : dense_plane_bytes(p, Np, Np);
}
// K chunks in flight per wave (prefetch depth); a row's K chunk count must be a
// multiple of it.
constexpr int dense_depth(Path p) { return (path_ebytes(p) == 1 && !path_fp4(p)) ? 4 : 2; }
// Spin padding of the dense paths: a multiple of 128 and of depth K chunks.
constexpr int dense_pad(Path p) {
    return path_kpc(p) * dense_depth(p) > 128 ? path_kpc(p) * dense_depth(p) : 128;
}
// m-blocks of 16 replicas per wave for C replica columns (workgroup covers
// 4 * 16 * mbw columns).
inline int dense_mbw(int C) { return C <= 64 ? 1 : C <= 128 ? 2 : 4; }

enum DenseEpilogue : int32_t { EPI_UPDATE = 0, EPI_FIELDS = 1 };

struct DenseStepArgs {
    int N, Np, R, C;
    int nkc;                        // K chunks of 128 bytes per row: dense_nkc(path, Np)
    int reverse;                    // traverse K chunks from the last one
    const uint8_t *J, *J_lo;        // fragment-tiled [Np/16][nkc]; J_lo: bf16 low part
    const uint8_t *g, *g_lo;        // operand f(X_n), fragment-tiled [Cg/16][nkc]
    uint8_t *g_next, *g_next_lo;    // operand f(X_{n+1}) (update epilogue)
    const float *h;                 // [Np], zero padded
    const float *x_in;              // [C][Np]
    float *x_out, *y;               // [C][Np]; y in place
    float *phi;                     // [C][Np] (fields epilogue)
    const float *jp;                // J_perp[r][n] at this step, run stride jp_stride
    int64_t jp_stride;
    StepCoef k;
    int fmode;
};

// One step of the dense path: Phi = J f(X_n) on MFMA for a workgroup tile of
// DENSE_TN spins x 64*mbw replica columns, then either the fused update
// (Eqs. 6-7, wall, next operand) or a plain store of Phi.
// grid = (Np / DENSE_TN, Cg / (64 * mbw)).
hipError_t launch_dense_step(Path path, DenseEpilogue epi, int mbw, int Cg, const DenseStepArgs &a,
                             hipStream_t st);

// ---- grouped steps of the serving loop ----------------------------------------
// Three-body terms (the cubic part of Eq. 11) of a CSR instance, listed per
// member spin: entries ptr[i]..ptr[i+1]-1 of spin i hold the other two
// members ab[2e], ab[2e+1] of each triple containing i (in the order the
// triples were given) and its weight k (float32; float64 copy k64 for the
// energies). ptr == nullptr: no three-body terms.
struct Tri3 {
    const int32_t *ptr = nullptr;
    const int32_t *ab = nullptr;
    const float *k = nullptr;
    const double *k64 = nullptr;
};

// One task per resident instance; the tasks of a group (same kernel
// specialisation) are stepped together by one grouped launch per step, a
// grid-stride loop over the virtual blocks of all tasks (task q owns blocks
// [first_block, first_block + nblocks)). Step n = n_base + offset runs while
// n < n_end; the state buffers ping-pong on the parity of n (x[n & 1] in).
struct GroupTask {
    int first_block, nblocks;
    int n_base, n_end;
    int S;                   // schedule length (J_perp row stride)
    int N, ld;               // spins; state row stride (CSR: Cs, dense: Np)
    int R, C;
    int nchunk;              // CSR: column chunks of the step; dense: spin tiles (Np / DENSE_TN)
    int nkc, fmode;
    float kB, dt, kD;
    float *x[2];
    float *y;
    void *g[2], *g_lo[2];
    const void *J, *J_lo;    // dense, fragment-tiled
    const int32_t *row_ptr, *col;
    const float *val;        // CSR
    Tri3 t3;                 // CSR three-body terms
    const float *h, *jp, *coefA, *delta;   // jp: [runs][S]; coefA [S]; delta [S+1]
};
struct GroupHeader {
    int ntask, total_blocks;
};
int csr_step_blocks(int N, int C);
int csr_step_chunks(int C);
bool csr_ring_shfl(int R);
hipError_t launch_group_csr(bool ballistic, bool shfl, const GroupHeader *hdr, const GroupTask *tasks, int grid,
                            int offset, hipStream_t st);
hipError_t launch_group_dense(Path path, int mbw, const GroupHeader *hdr, const GroupTask *tasks, int grid,
                              int offset, hipStream_t st);

// J in the contraction precision (fragment-tiled, groups of DENSE_TN/16 row
// blocks) from the zero-padded row-major float64 J64 [Np][Np].
hipError_t launch_convert_j(Path path, const double *J64, int Np, int nkc, void *Jd, void *Jd_lo, hipStream_t st);

// Bit-packed +-1 J (PATH_FP8PK / PATH_FP4PK) from row-major sign bits of the
// N x N matrix: words = ceil(N / 32) uint32 per row, bit j % 32 of word
// i * words + j / 32 set where J_ij < 0 (the diagonal clear).
hipError_t launch_convert_j_bits(Path path, const uint32_t *sign_bits, int N, int Np, int nkc, void *Jd,
                                 hipStream_t st);

// Operand f(X) (fragment-tiled, groups of mbw row blocks) from state [C][Np]
// with threshold delta.
hipError_t launch_dense_operand(Path path, int fmode, int N, int Np, int C, int nkc, int mbw, const float *x,
                                void *g, void *g_lo, float delta, hipStream_t st);

// CSR fused step over state [N][Cs] (spin-major): gathers of the operand
// (int8 f values, or x itself for ballistic f), pump/ring/kick/drift/wall,
// next operand with delta_next.
hipError_t launch_csr_step(int fmode, int N, int Cs, int R, int runs, const int32_t *row_ptr,
                           const int32_t *col, const float *val, const Tri3 &t3, const float *h,
                           const float *x_in, float *x_out, float *y, const int8_t *g_in,
                           int8_t *g_out, const float *jp, int64_t jp_stride, StepCoef k,
                           hipStream_t st);

// Register-resident CSR loop (K steps per launch, every workgroup
// co-resident); see kernels_resident.hip. Arrays are device pointers;
// NR = resident_rows(N) rows, rows N..NR-1 are zero padding.
struct ResidentArgs {
    int N, R, S, n0, K, fmode, nwg;
    const int32_t *colpad;  // [NR][D] neighbour indices (padding: index 0, weight 0)
    const float *valpad;    // [D][NR] weights, padded with 0
    const float *h;         // [NR]
    float *x, *y;           // ORDER_COLBLOCK8 [nwg][NR][8] state, updated in place
    const float *jp;        // [runs][S]
    const float *coefA;     // [S]   (a0 - a_n)/R
    const float *delta;     // [S+1] Delta_n
    float kB, dt, kD;
    float *xpub;            // [2][nwg][2][NR] published edge columns
    int *flags;             // [nwg] steps completed (monotonic)
    int *epoch_cnt;         // [nwg] launches started (monotonic)
    int epoch;              // this launch's number (>= 1)
    int *err;               // [1] set on a wait timeout
    uint8_t *sbits;         // [nwg][NR] sign bytes of the final state (bit k: column k negative)
};
int resident_degree(int maxdeg);        // padded degree D, or -1 when too large
size_t resident_lds_bytes(int N, int D);
int resident_cols();
int resident_rpt(int N);             // rows per thread, or -1 when N is too large
int resident_rows(int N);            // padded row count NR, or -1
int resident_threads(int N);         // threads per workgroup, or -1
hipError_t resident_max_blocks(int D, int N, int *blocks_per_cu);
// Raises a kernel's dynamic LDS limit on the current device to at least lds
// bytes. The runtime call is made only when the limit grows (one lookup under
// a mutex otherwise), so that launches do not pay for it every time.
hipError_t ensure_dyn_lds(const void *fn, size_t lds);
hipError_t launch_csr_resident(const ResidentArgs &a, int D, hipStream_t st);

// Resident loop for small dense instances (kernels_small.hip): one
// workgroup per run, K steps per launch, J float32 [N][N] row-major, state
// [C][Np] replica-major updated in place.
constexpr int SMALL_MAX_N = 128;
constexpr int SMALL_MAX_ELEMS = 4096;   // R * N
struct SmallArgs {
    int N, Np, R, S, n0, K, fmode;
    int jbits;            // every J entry is -1, 0 or +1: the bit-mask coupling sum may be used
    const float *J;       // [N][N]
    const float *h;       // [Np]
    float *x, *y;         // [C][Np]
    const float *jp;      // [runs][S]
    const float *coefA;   // [S]   (a0 - a_n)/R
    const float *delta;   // [S+1] Delta_n
    float kB, dt, kD;
};
size_t small_lds_bytes(int N, int R);
hipError_t launch_dense_small(const SmallArgs &a, int runs, hipStream_t st);

// CSR operand from state [N][Cs].
hipError_t launch_csr_operand(int fmode, int N, int Cs, int C, const float *x, int8_t *g,
                              float delta, hipStream_t st);

// CSR coupling sum phi[N][Cs] = J f(X) (test hook).
hipError_t launch_csr_fields(int fmode, int N, int Cs, int C, const int32_t *row_ptr,
                             const int32_t *col, const float *val, const Tri3 &t3, const float *x,
                             const int8_t *g, float *phi, hipStream_t st);

// Counter-based initial state: x, y ~ U[-amp, amp] from Philox4x32-10 keyed by
// seed, counter (i, c), i the caller's spin index: orig[row] when rows hold
// relabelled spins, else the row; element (i, c) at state_off(order, ld, i, c).
hipError_t launch_init_state(int N, int C, int order, int ld, uint64_t seed, double amp, const int32_t *orig,
                             float *x, float *y, hipStream_t st);

// Copy of an N x C float state from one order to another (rows of dst outside
// [0, N) are left as they are).
hipError_t launch_state_reorder(int N, int C, int order_in, int ld_in, const float *src, int order_out, int ld_out,
                                float *dst, hipStream_t st);

// Readout spins sign(x) (sign(0) = +1) as float64 +-1 into S[Cp][Np]
// (zero padding) from the state, for the energy GEMM.
hipError_t launch_readout_f64(int N, int Np, int C, int ld, bool spin_major, const float *x,
                              double *S, hipStream_t st);

// Row-major N x N float64 src into the first N columns of the rows of dst
// (row length Np >= N; the rest of dst is left as it is).
hipError_t launch_pad_rows(const double *src, int N, int Np, double *dst, hipStream_t st);
// bytes from device memory src to dst, the device address of pinned coherent
// host memory (both 16-byte aligned), written by the device over the bus
hipError_t launch_copy_to_host(const uint8_t *src, uint8_t *dst, size_t bytes, hipStream_t st);

// Spin rows [count][N] in the caller's order -> internal rows (row i holds the
// caller's spin orig[i]).
hipError_t launch_spins_to_rows(int N, int count, const int32_t *orig, const int8_t *in, int8_t *out, hipStream_t st);

// int8 spins [count][N] -> float64 S[Cp][Np].
hipError_t launch_spins_to_f64(int N, int Np, int count, const int8_t *spins, double *S,
                               hipStream_t st);

// E[c] = sum_i s_ci (-1/2 sum_z phis[z][c][i] - h_i), fixed-order reduction.
hipError_t launch_energy_reduce(int N, int Np, int count, int Cp, int splits,
                                const double *phis, const double *S, const double *h,
                                double *E, hipStream_t st);

// CSR energies of the readout of x (element (i, c) at state_off(order, ld, i, c))
// or of given spins. The state energies are summed in one fixed order: per
// column, row blocks of rpb = ceil(N / nblk_rows) rows, each summed in row
// order (neighbours in CSR order); row block rb added into slot
// rb % ENERGY_SLOTS in increasing rb; then a pairwise tree over the slots
// (slot t += slot t + w for w = ENERGY_SLOTS/2, ..., 1). nblk_rows >=
// ENERGY_SLOTS unless N is smaller, so that every slot can be one thread's.
constexpr int ENERGY_SLOTS = 1024;
hipError_t launch_csr_energy_state(int N, int order, int ld, int C, const int32_t *row_ptr,
                                   const int32_t *col, const double *val, const Tri3 &t3, const double *h,
                                   const float *x, double *partial, int nblk_rows, double *E,
                                   hipStream_t st);
// The same energies of a column-block state (ORDER_COLBLOCK8 with leading
// dimension ld >= N, C % 8 == 0, N * 8 bytes of LDS, even D, no three-body
// terms), equal bit for bit. The couplings of row block rb (rows rb*rpb ..
// rb*rpb + rpb - 1, the row blocks of the spin-major energies: nrb * rpb >= N)
// are stored row block innermost: rcol / rval [RS][D][nrb] (neighbours in CSR
// order, then index 0 with weight 0), rh [RS][nrb] (h, 0 past N), with
// RS = energy_colblock_rows(rpb). sbits: the sign bytes the resident loop
// wrote for this same x ([C/8][ld], bit k: column k negative), read in place
// of x's 32 bytes per row and block; nullptr: the signs are taken from x.
int energy_colblock_rows(int rpb);
hipError_t launch_csr_energy_colblock(int N, int ld, int C, int D, int nrb, int rpb, const int32_t *rcol,
                                      const double *rval, const double *rh, const float *x,
                                      const uint8_t *sbits, double *E, hipStream_t st);
// The same energies followed by the readout of a run, in one launch: the best
// update of launch_best_update (without the copy of x's spins, which are taken
// from sbits or x as above) by the last workgroup of each run to finish, which
// then writes the run's best energy and best spins straight into the pinned
// host readout block (host: its device address; layout best energies
// [runs] float64, the error word at byte 8*runs, best spins [runs][N] at
// byte 8*runs + 8), and workgroup 0 copies the error word err there. cnt:
// [runs] arrival counters, zero before the launch and left zero after it.
// R % 8 == 0, C == R * runs, ld % 8 == 0.
struct ReadoutFuse {
    int R = 0, runs = 0;
    double *best_E = nullptr;
    int64_t *best_step = nullptr;
    int8_t *best_spins = nullptr;
    const int *err = nullptr;
    int *cnt = nullptr;
    uint8_t *host = nullptr;
    int64_t step = 0;
    int reset = 0;
};
hipError_t launch_csr_readout_colblock(int N, int ld, int C, int D, int nrb, int rpb, const int32_t *rcol,
                                       const double *rval, const double *rh, const float *x,
                                       const uint8_t *sbits, double *E, const ReadoutFuse &f, hipStream_t st);
hipError_t launch_csr_energy_spins(int N, int count, const int32_t *row_ptr, const int32_t *col,
                                   const double *val, const Tri3 &t3, const double *h, const int8_t *spins,
                                   double *E, hipStream_t st);

// Exact energies of the readout of a dense state [C][Np] whose J is integral
// (fp8 / int8 paths): the readout operand sign(x) (sign(0) = +1, padded spins
// 0) in the fragment-tiled layout, contracted by the dense step's fields
// epilogue into phi [C][Np], then E_c = -1/2 s.phi - h.s in float64.
hipError_t launch_readout_operand(Path path, int N, int Np, int C, int nkc, int mbw, const float *x, void *g,
                                  hipStream_t st);
hipError_t launch_energy_fields(int N, int Np, int C, const float *x, const float *phi, const double *h, double *E,
                                hipStream_t st);

// Per-run best over replicas with tie -> lowest k; updates best_E/best_step
// when strictly lower (than +inf when reset: the previous best is discarded)
// and copies the winning readout spins; one launch, one workgroup per run.
// Above BEST_SPLIT_N spins the update runs as two launches (selection, then
// the spin copy over many workgroups) with sel [runs] int scratch; the
// results are the same.
constexpr int BEST_SPLIT_N = 32768;
hipError_t launch_best_update(int N, int R, int runs, int order, int ld, const float *x, const double *E,
                              double *best_E, int64_t *best_step, int8_t *best_spins, int64_t step, bool reset,
                              int *sel, hipStream_t st);

}  // namespace sbqa
