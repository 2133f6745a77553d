// Initial state, readout, energies and best-solution selection for gfx950.
//   * Initial state: x, y ~ U[-amp, amp] (random start, Sec. II.A) from the
//     counter-based Philox4x32-10 generator (Salmon et al., SC'11), keyed by
//     the seed and counted by (i, c), so the draw is layout-independent.
//   * Energies E(s) = -1/2 s^T J s - h^T s of readouts s = sign(x) (sign(0) =
//     +1) in float64 with fixed-order reductions (exact for integer J, h).
//   * Best per run over its R replicas (Sec. II.B), ties -> lowest replica,
//     earlier evaluations kept on equal energy.
#include "sbqa_internal.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

namespace sbqa {
namespace {

// Philox4x32 round constants (multipliers and Weyl key increments).
constexpr uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 ctr, uint2 key) {
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd > 0) {
            key.x += PHILOX_W0;
            key.y += PHILOX_W1;
        }
        const uint64_t p0 = (uint64_t)PHILOX_M0 * ctr.x;
        const uint64_t p1 = (uint64_t)PHILOX_M1 * ctr.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        ctr = make_uint4(hi1 ^ ctr.y ^ key.x, lo1, hi0 ^ ctr.w ^ key.y, lo0);
    }
    return ctr;
}

// u in [0, 1) with 24 random bits, then amp*(2u - 1) in float64 rounded once.
__device__ __forceinline__ float uniform_sym(uint32_t bits, double amp) {
    const double u = (double)(bits >> 8) * (1.0 / 16777216.0);
    return (float)(amp * (2.0 * u - 1.0));
}

__global__ void k_init_state(int N, int C, int order, int ld, uint32_t key_lo, uint32_t key_hi,
                             double amp, const int32_t *__restrict__ orig, float *__restrict__ x,
                             float *__restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * C) return;
    const int i = (int)(e / C), c = (int)(e % C);
    // the counter is the caller's spin index (row i holds spin orig[i] when
    // the spins are relabelled internally)
    const uint32_t si = orig ? (uint32_t)orig[i] : (uint32_t)i;
    const uint4 r = philox4x32_10(make_uint4(si, (uint32_t)c, 0u, 0u), make_uint2(key_lo, key_hi));
    const int64_t o = state_off(order, ld, i, c);
    x[o] = uniform_sym(r.x, amp);
    y[o] = uniform_sym(r.y, amp);
}

__global__ void k_state_reorder(int N, int C, int order_in, int ld_in, const float *__restrict__ src,
                                int order_out, int ld_out, float *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * C) return;
    const int i = (int)(e / C), c = (int)(e % C);
    dst[state_off(order_out, ld_out, i, c)] = src[state_off(order_in, ld_in, i, c)];
}

__global__ void k_readout_f64(int N, int Np, int C, int ld, int spin_major, const float *__restrict__ x,
                              double *__restrict__ S) {
    const int c = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Np) return;
    double s = 0.0;
    if (i < N && c < C) {
        const float v = spin_major ? x[(int64_t)i * ld + c] : x[(int64_t)c * ld + i];
        s = v >= 0.0f ? 1.0 : -1.0;
    }
    S[(int64_t)c * Np + i] = s;
}

__global__ void k_spins_to_f64(int N, int Np, int count, const int8_t *__restrict__ spins, double *__restrict__ S) {
    const int m = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Np) return;
    S[(int64_t)m * Np + i] = (i < N && m < count) ? (double)spins[(int64_t)m * N + i] : 0.0;
}

// Block per configuration; per-thread strided sums, then a fixed LDS tree.
__global__ __launch_bounds__(256) void k_energy_reduce(int N, int Np, int Cp, int splits,
                                                       const double *__restrict__ phis,
                                                       const double *__restrict__ S,
                                                       const double *__restrict__ h, double *__restrict__ E) {
    __shared__ double sq[256], sl[256];
    const int c = blockIdx.x, t = threadIdx.x;
    double q = 0.0, l = 0.0;
    for (int i = t; i < N; i += 256) {
        double phi = phis[(int64_t)c * Np + i];
        for (int z = 1; z < splits; ++z) phi += phis[((int64_t)z * Cp + c) * Np + i];
        const double s = S[(int64_t)c * Np + i];
        q += s * phi;
        if (h) l += h[i] * s;
    }
    sq[t] = q;
    sl[t] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sq[t] += sq[t + w];
            sl[t] += sl[t + w];
        }
        __syncthreads();
    }
    if (t == 0) E[c] = -0.5 * sq[0] - sl[0];
}

// Energies from exact integer fields Phi = J s of the readout s = sign(x)
// (sign(0) = +1), replica-major [C][Np]: E_c = -1/2 sum_i s_ci Phi_ci -
// sum_i h_i s_ci, block per column, the same fixed-order reduction as
// k_energy_reduce (every partial sum an integer for integer J and h).
__global__ __launch_bounds__(256) void k_energy_fields(int N, int Np, const float *__restrict__ x,
                                                       const float *__restrict__ phi, const double *__restrict__ h,
                                                       double *__restrict__ E) {
    __shared__ double sq[256], sl[256];
    const int c = blockIdx.x, t = threadIdx.x;
    double q = 0.0, l = 0.0;
    for (int i = t; i < N; i += 256) {
        const double s = x[(int64_t)c * Np + i] >= 0.0f ? 1.0 : -1.0;
        q += s * (double)phi[(int64_t)c * Np + i];
        if (h) l += h[i] * s;
    }
    sq[t] = q;
    sl[t] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sq[t] += sq[t + w];
            sl[t] += sl[t + w];
        }
        __syncthreads();
    }
    if (t == 0) E[c] = -0.5 * sq[0] - sl[0];
}

// Three-body part of the energy of one spin i, as s_i psi_i with psi_i the
// sum over the triples containing i of K s_a s_b; summed over i this counts
// every triple three times (E3 = -1/3 sum_i s_i psi_i, exact for integer K).
template <class SpinOf>
__device__ __forceinline__ double tri_psi(const Tri3 &t3, int i, SpinOf spin) {
    double psi = 0.0;
    for (int p = t3.ptr[i]; p < t3.ptr[i + 1]; ++p) psi += t3.k64[p] * (spin(t3.ab[2 * p]) * spin(t3.ab[2 * p + 1]));
    return psi;
}

// CSR energies of the readout of a state (element (i, c) at
// state_off(order, ld, i, c)). Stage 1: block (row block rb, up to 256
// columns) accumulates per column over its rows in row order.
__global__ __launch_bounds__(256) void k_csr_energy_partial(int N, int order, int ld, int C, int rows_per_blk,
                                                            const int32_t *__restrict__ row_ptr,
                                                            const int32_t *__restrict__ col,
                                                            const double *__restrict__ val, const Tri3 t3,
                                                            const double *__restrict__ h,
                                                            const float *__restrict__ x,
                                                            double *__restrict__ partial) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int rb = blockIdx.y;
    if (c >= C) return;
    double q = 0.0, l = 0.0, q3 = 0.0;
    auto spin = [&](int j) { return x[state_off(order, ld, j, c)] >= 0.0f ? 1.0 : -1.0; };
    const int i0 = rb * rows_per_blk, i1 = min(N, i0 + rows_per_blk);
    for (int i = i0; i < i1; ++i) {
        double phi = 0.0;
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const float xv = x[state_off(order, ld, col[p], c)];
            phi += val[p] * (xv >= 0.0f ? 1.0 : -1.0);
        }
        const double s = x[state_off(order, ld, i, c)] >= 0.0f ? 1.0 : -1.0;
        q += s * phi;
        if (h) l += h[i] * s;
        if (t3.ptr) q3 += s * tri_psi(t3, i, spin);
    }
    partial[((int64_t)rb * C + c) * 3] = q;
    partial[((int64_t)rb * C + c) * 3 + 1] = l;
    partial[((int64_t)rb * C + c) * 3 + 2] = q3;
}

// The pairwise tree over ENERGY_SLOTS = 1024 slots (slot t += slot t + w for
// w = 512, 256, ..., 1) reduced by one wave in registers: lane ln holds slots
// ln + 64 j (j < 16); the levels of width 512 .. 64 add register
// j + width / 64 into j, the levels 32 .. 1 add lane ln + width into lane
// ln, so every level adds the same pairs, left + right, as the slot-by-slot
// tree. Lane 0 returns the sum of src[0 .. 1023].
__device__ __forceinline__ double wave_tree1024(const double *src, int ln) {
    static_assert(ENERGY_SLOTS == 1024, "16 slots per lane of a 64-lane wave");
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = src[ln + 64 * j] + src[ln + 64 * (j + 8)];
#pragma unroll
    for (int wd = 4; wd >= 1; wd >>= 1)
#pragma unroll
        for (int j = 0; j < wd; ++j) v[j] = v[j] + v[j + wd];
    double x = v[0];
#pragma unroll
    for (int s2 = 32; s2 >= 1; s2 >>= 1) {
        const double o = __shfl_down(x, s2);
        if (ln < s2) x = x + o;
    }
    return x;
}

// Stage 2: block per column, thread t sums the row blocks of slot t in
// increasing order, then the pairwise tree over the slots.
__global__ __launch_bounds__(ENERGY_SLOTS) void k_csr_energy_final(int C, int nrb, const double *__restrict__ partial,
                                                                   double *__restrict__ E) {
    __shared__ double sq[ENERGY_SLOTS], sl[ENERGY_SLOTS], s3[ENERGY_SLOTS];
    const int c = blockIdx.x, t = threadIdx.x;
    double q = 0.0, l = 0.0, q3 = 0.0;
    for (int rb = t; rb < nrb; rb += ENERGY_SLOTS) {
        q += partial[((int64_t)rb * C + c) * 3];
        l += partial[((int64_t)rb * C + c) * 3 + 1];
        q3 += partial[((int64_t)rb * C + c) * 3 + 2];
    }
    sq[t] = q;
    sl[t] = l;
    s3[t] = q3;
    __syncthreads();
    // the pairwise tree of each sum, by waves 0, 1 and 2
    __shared__ double red[3];
    const int u = t >> 6;
    if (u < 3) {
        const double x = wave_tree1024(u == 0 ? sq : u == 1 ? sl : s3, t & 63);
        if ((t & 63) == 0) red[u] = x;
    }
    __syncthreads();
    if (t == 0) E[c] = -0.5 * red[0] - red[1] - red[2] / 3.0;
}

// CSR energies of the readout of a column-block state (ORDER_COLBLOCK8, no
// three-body terms), one workgroup of ENERGY_SLOTS threads per block of 8
// columns. The sums are those of k_csr_energy_partial + k_csr_energy_final,
// in the same order: per column, row blocks of rpb rows summed in row order
// (neighbours in CSR order), row block rb added by thread rb % ENERGY_SLOTS
// in increasing rb, then the same pairwise tree; so the energies equal those
// of a spin-major context bit for bit. The block's signs go to LDS once, 8
// bytes per row (byte k: 0x80 when column k is negative, sign(0) = +1); a
// term s_j J_ij, or s_i phi_i, is its float64 operand with the high word
// xor-ed by the row's byte k moved to the top (one byte permute), exactly the
// product by +-1. The couplings are stored with the row block innermost
// ([RS][D][nrb] column indices and float64 weights, padding index 0 with
// weight 0: a zero term leaves the sum unchanged; [RS][nrb] fields h, 0 past
// N), so that the threads of a wave, which take consecutive row blocks, read
// consecutive words (a run per row block put every lane on its own cache
// lines).
__device__ __forceinline__ double flip_sign(double v, uint32_t mask) {
    return __hiloint2double(__double2hiint(v) ^ (int)mask, __double2loint(v));
}
// byte k (0..3) of w at the top of a word, the rest zero
__device__ __forceinline__ uint32_t byte_to_top(uint32_t w, int k) {
    return __builtin_amdgcn_perm(w, w, ((uint32_t)k << 24) | 0x000C0C0Cu);
}
// 8 sign bits (bit k: column k) as 8 bytes (0x80 per set bit)
__device__ __forceinline__ uint2 spread_signs(uint32_t b) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lo |= ((b >> k) & 1u) << (8 * k + 7);
        hi |= ((b >> (k + 4)) & 1u) << (8 * k + 7);
    }
    return make_uint2(lo, hi);
}

// Best of run r (Sec. II.B), by the first wavefront of a workgroup (t < 64):
// the argmin over the run's R energies (tie -> lowest k), reduced across
// lanes; the stored best (+inf when reset) is replaced only when strictly
// lower. Thread 0 sets *sel to the winning replica, or -1 when the stored best
// stays, and *kept to the stored best energy after the update. The comparison
// is kept in vector registers on purpose: a wave-uniform float64 compare
// feeding a scalar select was observed to be lowered with a stale condition
// code on gfx950. AGENT: the energies were written by other workgroups of the
// same launch (coherent loads).
template <bool AGENT>
__device__ __forceinline__ void select_best(const double *E, int r, int R, int t, double *best_E, int64_t *best_step,
                                            int64_t step, int reset, int *sel, double *kept) {
    if (t >= 64) return;
    double eb = INFINITY;
    int kb = 0x7FFFFFFF;
    for (int k = t; k < R; k += 64) {
        const double *ep = E + (int64_t)r * R + k;
        const double e = AGENT ? __hip_atomic_load(const_cast<double *>(ep), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : *ep;
        if (e < eb) { eb = e; kb = k; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double eo = __shfl_xor(eb, off);
        const int ko = __shfl_xor(kb, off);
        const bool take = (eo < eb) || (eo == eb && ko < kb);
        eb = take ? eo : eb;
        kb = take ? ko : kb;
    }
    const double stored = best_E[r];
    const double cur = reset ? INFINITY : stored;
    const int better = (eb < cur) ? 1 : 0;
    if (t == 0) {
        *sel = better ? kb : -1;
        *kept = better ? eb : stored;
        if (better) {
            best_E[r] = eb;
            best_step[r] = step;
        }
    }
}

template <int D, bool FUSE>
__global__ __launch_bounds__(ENERGY_SLOTS) void k_csr_energy_colblock(int N, int ld, int nrb, int rpb, int RS,
                                                                      const int32_t *__restrict__ rcol,
                                                                      const double *__restrict__ rval,
                                                                      const double *__restrict__ rh,
                                                                      const float *__restrict__ x,
                                                                      const uint8_t *__restrict__ sbits,
                                                                      double *__restrict__ E, const ReadoutFuse f) {
    constexpr int T = ENERGY_SLOTS;
    // rows whose loads are issued together, neighbours per group of loads
    // (within 128 registers per lane)
    constexpr int RB = D <= 4 ? 2 : 1;
    constexpr int G = D <= 8 ? D : 4;
    static_assert(D % G == 0, "whole neighbour groups");
    extern __shared__ __align__(16) uint8_t smem[];
    uint2 *sm = reinterpret_cast<uint2 *>(smem);   // [N]: sign bytes of columns 0-3, 4-7
    const int w = blockIdx.x, t = threadIdx.x;
    const float *xb = x + (int64_t)w * ld * 8;
    // sign bytes: 16 rows per thread and load
    for (int base = 0; sbits && base < N; base += T * 16) {
        const int i0 = base + 16 * t;
        if (i0 >= N) continue;
        const uint8_t *sb = sbits + (int64_t)w * ld + i0;
        uint4 v;
        if (i0 + 16 <= N) v = *reinterpret_cast<const uint4 *>(sb);
        else {
            uint32_t wv[4] = {0u, 0u, 0u, 0u};
            for (int u = 0; i0 + u < N; ++u) wv[u / 4] |= (uint32_t)sb[u] << (8 * (u % 4));
            v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
        }
        const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = i0 + u;
            if (i < N) sm[i] = spread_signs((vw[u / 4] >> (8 * (u % 4))) & 0xFFu);
        }
    }
    // from x: 4 rows per thread in flight (one round trip for N <= 4096)
    auto sbyte = [](float v, int k) { return (v < 0.0f ? 0x80u : 0u) << (8 * k); };
    for (int base = 0; !sbits && base < N; base += T * 4) {
        float4 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = min(base + u * T + t, N - 1);
            a[u] = *reinterpret_cast<const float4 *>(xb + (int64_t)i * 8);
            b[u] = *reinterpret_cast<const float4 *>(xb + (int64_t)i * 8 + 4);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * T + t;
            if (i < N)
                sm[i] = make_uint2(sbyte(a[u].x, 0) | sbyte(a[u].y, 1) | sbyte(a[u].z, 2) | sbyte(a[u].w, 3),
                                   sbyte(b[u].x, 0) | sbyte(b[u].y, 1) | sbyte(b[u].z, 2) | sbyte(b[u].w, 3));
        }
    }
    __syncthreads();
    double q[8], l[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = l[k] = 0.0;
    for (int rb = t; rb < nrb; rb += T) {
        double pq[8], pl[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) pq[k] = pl[k] = 0.0;
        const int i0 = rb * rpb, nrow = min(N - i0, rpb);
        for (int jb = 0; jb < nrow; jb += RB) {
            double hv[RB];
            // rows past the block's end: their run's padding (RS >= rpb
            // rounded up to RB), discarded below
#pragma unroll
            for (int r = 0; r < RB; ++r) hv[r] = rh[(uint32_t)((jb + r) * nrb + rb)];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const bool valid = jb + r < nrow;
                double phi[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) phi[k] = 0.0;
                // neighbours in groups of G (all of them for D <= 8): a
                // group's loads in flight together
#pragma unroll
                for (int p0 = 0; p0 < D; p0 += G) {
                    int cj[G];
                    double vj[G];
#pragma unroll
                    for (int e = 0; e < G; ++e) {
                        const uint32_t o = (uint32_t)(((jb + r) * D + p0 + e) * nrb + rb);   // < 2^31
                        cj[e] = rcol[o];
                        vj[e] = rval[o];
                    }
#pragma unroll
                    for (int p = 0; p < G; ++p) {
                        const uint2 m = sm[cj[p]];
                        const double v = vj[p];
#pragma unroll
                        for (int k = 0; k < 8; ++k) phi[k] += flip_sign(v, byte_to_top(k < 4 ? m.x : m.y, k & 3));
                    }
                }
                const uint2 m = sm[i0 + min(jb + r, nrow - 1)];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t mk = byte_to_top(k < 4 ? m.x : m.y, k & 3);
                    const double nq = pq[k] + flip_sign(phi[k], mk), nl = pl[k] + flip_sign(hv[r], mk);
                    pq[k] = valid ? nq : pq[k];
                    pl[k] = valid ? nl : pl[k];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            q[k] += pq[k];
            l[k] += pl[k];
        }
    }
    __syncthreads();   // the signs are dead: their LDS holds the reduction
    double *sq = reinterpret_cast<double *>(smem), *sl = sq + 8 * T;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        sq[k * T + t] = q[k];
        sl[k * T + t] = l[k];
    }
    __syncthreads();
    // the pairwise tree of each of the 16 sums (q and l of 8 columns), one
    // wave each
    static_assert(T == 1024, "16 waves, one sum each");
    __shared__ double red[16];
    {
        const int u = t >> 6;
        const double x = wave_tree1024(u < 8 ? sq + u * T : sl + (u - 8) * T, t & 63);
        if ((t & 63) == 0) red[u] = x;
    }
    __syncthreads();
    const double s3 = 0.0;   // no three-body terms on this path
    if constexpr (!FUSE) {
        if (t < 8) E[w * 8 + t] = -0.5 * red[t] - red[8 + t] - s3 / 3.0;
    } else {
        // the best update of the run and the readout block, by the last of
        // the run's R / 8 workgroups to finish its energies: they are stored
        // coherently for the device and completed before the run's arrival
        // counter is raised; the last one reads them after it (and sets the
        // counter back to zero for the next launch)
        __shared__ int last, sel;
        __shared__ double kept;
        if (t < 8)
            __hip_atomic_store(E + w * 8 + t, -0.5 * red[t] - red[8 + t] - s3 / 3.0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (w == 0 && t == 0) *reinterpret_cast<int *>(f.host + (size_t)8 * f.runs) = *f.err;
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int P = f.R / 8, run = w / P;
        if (t == 0) {
            const int old = __hip_atomic_fetch_add(f.cnt + run, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = old == P - 1;
            if (last) __hip_atomic_store(f.cnt + run, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (!last) return;
        select_best<true>(E, run, f.R, t, f.best_E, f.best_step, f.step, f.reset, &sel, &kept);
        __syncthreads();
        if (t == 0) reinterpret_cast<double *>(f.host)[run] = kept;
        // spins of the winner (sign(0) = +1) to the device best and the host
        // block, or the stored best spins to the host block; 8 rows a thread
        const int k = sel;
        int8_t *dev = f.best_spins + (int64_t)run * N;
        int8_t *hst = reinterpret_cast<int8_t *>(f.host + (size_t)8 * f.runs + 8) + (int64_t)run * N;
        const int c = run * f.R + k, wb = c >> 3, kk = c & 7;
        for (int i0 = 8 * t; i0 < N; i0 += 8 * T) {
            int8_t v[8];
            if (k < 0) {
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = i0 + u < N ? dev[i0 + u] : 0;
            } else if (sbits) {
                // rows up to ld are in the buffer (ld >= N, a multiple of 16)
                const uint2 b = *reinterpret_cast<const uint2 *>(sbits + (int64_t)wb * ld + i0);
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = (((u < 4 ? b.x : b.y) >> (8 * (u & 3) + kk)) & 1u) ? -1 : 1;
            } else {
                // rows up to ld are in the state (zero past N)
                const float *xw = x + ((int64_t)wb * ld + i0) * 8 + kk;
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = xw[u * 8] >= 0.0f ? 1 : -1;
            }
            // dev and hst have the same offset from 256-byte aligned bases
            if (i0 + 8 <= N && ((uintptr_t)(dev + i0) & 7u) == 0) {
                uint2 pk = make_uint2(0u, 0u);
#pragma unroll
                for (int u = 0; u < 8; ++u) (u < 4 ? pk.x : pk.y) |= (uint32_t)(uint8_t)v[u] << (8 * (u & 3));
                if (k >= 0) *reinterpret_cast<uint2 *>(dev + i0) = pk;
                *reinterpret_cast<uint2 *>(hst + i0) = pk;
            } else {
                for (int u = 0; u < 8 && i0 + u < N; ++u) {
                    if (k >= 0) dev[i0 + u] = v[u];
                    hst[i0 + u] = v[u];
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_csr_energy_spins(int N, const int32_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ val, const Tri3 t3,
                                                          const double *__restrict__ h,
                                                          const int8_t *__restrict__ spins, double *__restrict__ E) {
    __shared__ double sq[256], sl[256], s3[256];
    const int m = blockIdx.x, t = threadIdx.x;
    const int8_t *s = spins + (int64_t)m * N;
    auto spin = [&](int j) { return (double)s[j]; };
    double q = 0.0, l = 0.0, q3 = 0.0;
    for (int i = t; i < N; i += 256) {
        double phi = 0.0;
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) phi += val[p] * (double)s[col[p]];
        q += (double)s[i] * phi;
        if (h) l += h[i] * (double)s[i];
        if (t3.ptr) q3 += (double)s[i] * tri_psi(t3, i, spin);
    }
    sq[t] = q;
    sl[t] = l;
    s3[t] = q3;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sq[t] += sq[t + w];
            sl[t] += sl[t + w];
            s3[t] += s3[t + w];
        }
        __syncthreads();
    }
    if (t == 0) E[m] = -0.5 * sq[0] - sl[0] - s3[0] / 3.0;
}

// One workgroup per run: the best update of select_best, then the whole
// workgroup copies the winner's readout spins (sign(0) = +1).
__global__ __launch_bounds__(1024) void k_best_update(int N, int R, int order, int ld, const float *__restrict__ x,
                                                     const double *__restrict__ E, double *__restrict__ best_E,
                                                     int64_t *__restrict__ best_step,
                                                     int8_t *__restrict__ best_spins, int64_t step, int reset) {
    __shared__ int sel;
    __shared__ double kept;
    const int r = blockIdx.x, t = threadIdx.x;
    select_best<false>(E, r, R, t, best_E, best_step, step, reset, &sel, &kept);
    __syncthreads();
    const int k = sel;
    if (k < 0) return;
    const int c = r * R + k;
    for (int i = t; i < N; i += 1024) best_spins[(int64_t)r * N + i] = x[state_off(order, ld, i, c)] >= 0.0f ? 1 : -1;
}

// The same update in two launches, so that the spin copy of a large
// instance runs on many workgroups: k_best_select (one wave per run) writes
// the winning replica, or -1, to sel[r]; k_best_copy (runs x chunks) copies
// the winner's spins.
__global__ __launch_bounds__(64) void k_best_select(int R, const double *__restrict__ E, double *__restrict__ best_E,
                                                   int64_t *__restrict__ best_step, int *__restrict__ sel, int64_t step,
                                                   int reset) {
    __shared__ int s;
    __shared__ double kept;
    select_best<false>(E, blockIdx.x, R, threadIdx.x, best_E, best_step, step, reset, &s, &kept);
    __syncthreads();
    if (threadIdx.x == 0) sel[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_best_copy(int N, int R, int order, int ld, const float *__restrict__ x,
                                                  const int *__restrict__ sel, int8_t *__restrict__ best_spins) {
    const int r = blockIdx.y, k = sel[r];
    if (k < 0) return;
    const int c = r * R + k;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256)
        best_spins[(int64_t)r * N + i] = x[state_off(order, ld, i, c)] >= 0.0f ? 1 : -1;
}

// Row-major N x N float64 rows into the first N columns of rows of length Np.
// Whole 16-byte vectors, then the tail bytes one by one (thread 0).
__global__ void k_copy_to_host(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst, size_t bytes) {
    const size_t nv = bytes / 16;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nv; q += (size_t)gridDim.x * blockDim.x)
        reinterpret_cast<uint4 *>(dst)[q] = reinterpret_cast<const uint4 *>(src)[q];
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (size_t b = nv * 16; b < bytes; ++b) dst[b] = src[b];
}

__global__ void k_pad_rows(const double *__restrict__ src, int N, int Np, double *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    const int64_t i = e / N, j = e - i * N;
    dst[i * Np + j] = src[e];
}

// Spin rows from the caller's spin order to the internal rows: row i holds the
// caller's spin orig[i].
__global__ void k_spins_to_rows(int N, int count, const int32_t *__restrict__ orig, const int8_t *__restrict__ in,
                                int8_t *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * count) return;
    const int64_t m = e / N;
    const int i = (int)(e - m * N);
    out[e] = in[m * N + orig[i]];
}

}  // namespace

hipError_t launch_copy_to_host(const uint8_t *src, uint8_t *dst, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return hipErrorInvalidValue;
    const size_t n16 = (bytes + 15) / 16;
    const int blocks = (int)std::min<size_t>((n16 + 255) / 256, 1024);
    hipLaunchKernelGGL(k_copy_to_host, dim3(blocks), dim3(256), 0, st, src, dst, bytes);
    return hipGetLastError();
}

hipError_t launch_pad_rows(const double *src, int N, int Np, double *dst, hipStream_t st) {
    const int64_t n = (int64_t)N * N;
    if (Np < N) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, N, Np, dst);
    return hipGetLastError();
}

hipError_t launch_spins_to_rows(int N, int count, const int32_t *orig, const int8_t *in, int8_t *out, hipStream_t st) {
    const int64_t n = (int64_t)N * count;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spins_to_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, count, orig, in, out);
    return hipGetLastError();
}

hipError_t launch_init_state(int N, int C, int order, int ld, uint64_t seed, double amp, const int32_t *orig,
                             float *x, float *y, hipStream_t st) {
    const int64_t n = (int64_t)N * C;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_init_state, grid, block, 0, st, N, C, order, ld, (uint32_t)seed, (uint32_t)(seed >> 32), amp,
                       orig, x, y);
    return hipGetLastError();
}

hipError_t launch_state_reorder(int N, int C, int order_in, int ld_in, const float *src, int order_out, int ld_out,
                                float *dst, hipStream_t st) {
    const int64_t n = (int64_t)N * C;
    if (n == 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_state_reorder, grid, block, 0, st, N, C, order_in, ld_in, src, order_out, ld_out, dst);
    return hipGetLastError();
}

hipError_t launch_readout_f64(int N, int Np, int C, int ld, bool spin_major, const float *x, double *S,
                              hipStream_t st) {
    // S has Cp >= C rows; rows c >= C are written as zero by the grid below.
    const int Cp = (C + GEMM_BM - 1) / GEMM_BM * GEMM_BM;
    dim3 grid((Np + 255) / 256, Cp), block(256);
    hipLaunchKernelGGL(k_readout_f64, grid, block, 0, st, N, Np, C, ld, spin_major ? 1 : 0, x, S);
    return hipGetLastError();
}

hipError_t launch_spins_to_f64(int N, int Np, int count, const int8_t *spins, double *S, hipStream_t st) {
    const int Cp = (count + GEMM_BM - 1) / GEMM_BM * GEMM_BM;
    dim3 grid((Np + 255) / 256, Cp), block(256);
    hipLaunchKernelGGL(k_spins_to_f64, grid, block, 0, st, N, Np, count, spins, S);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(int N, int Np, int count, int Cp, int splits, const double *phis, const double *S,
                                const double *h, double *E, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_reduce, dim3(count), dim3(256), 0, st, N, Np, Cp, splits, phis, S, h, E);
    return hipGetLastError();
}

hipError_t launch_csr_energy_state(int N, int order, int ld, int C, const int32_t *row_ptr, const int32_t *col,
                                   const double *val, const Tri3 &t3, const double *h, const float *x,
                                   double *partial, int nblk_rows, double *E, hipStream_t st) {
    const int rows_per_blk = (N + nblk_rows - 1) / nblk_rows;
    // whole waves over the columns, at most 256 threads
    const int bx = std::min(256, (C + 63) / 64 * 64);
    dim3 grid((C + bx - 1) / bx, nblk_rows), block(bx);
    hipLaunchKernelGGL(k_csr_energy_partial, grid, block, 0, st, N, order, ld, C, rows_per_blk, row_ptr, col, val, t3,
                       h, x, partial);
    hipLaunchKernelGGL(k_csr_energy_final, dim3(C), dim3(ENERGY_SLOTS), 0, st, C, nblk_rows, partial, E);
    return hipGetLastError();
}

hipError_t ensure_dyn_lds(const void *fn, size_t lds) {
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> limit;   // (kernel, device) -> limit set
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    size_t &cur = limit[{fn, dev}];
    if (lds <= cur) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) cur = lds;
    return e;
}

// rows of a row block in the coupling copy: rpb rounded up to the kernel's
// batch of rows (2)
int energy_colblock_rows(int rpb) { return (rpb + 1) / 2 * 2; }

template <bool FUSE>
static hipError_t colblock_launch(int N, int ld, int C, int D, int nrb, int rpb, const int32_t *rcol,
                                  const double *rval, const double *rh, const float *x, const uint8_t *sbits,
                                  double *E, const ReadoutFuse &f, hipStream_t st) {
    const size_t lds = std::max<size_t>((size_t)N * 8, 2 * 8 * (size_t)ENERGY_SLOTS * sizeof(double));
    // even D: a batch of 8 rows is whole 16-byte vectors, and so is every row block's run
    // sign bytes are read 16 rows at a time: a 16-byte aligned row stride
    const int RS = energy_colblock_rows(rpb);
    // the kernel indexes the coupling copy with 32-bit offsets
    if (C % 8 || ld < N || (int64_t)nrb * rpb < N || lds > 160 * 1024 || D % 2 || (sbits && ld % 16) ||
        (int64_t)RS * D * nrb >= ((int64_t)1 << 31))
        return hipErrorInvalidValue;
    // fused readout: whole 8-column blocks per run, rows up to a multiple of 8
    // readable in the state (ld % 8 == 0), every buffer present
    if (FUSE && (f.R <= 0 || f.R % 8 || f.runs <= 0 || (int64_t)f.R * f.runs != C || ld % 8 || !f.best_E ||
                 !f.best_step || !f.best_spins || !f.err || !f.cnt || !f.host || ((uintptr_t)f.host & 7u)))
        return hipErrorInvalidValue;
    const dim3 grid(C / 8), block(ENERGY_SLOTS);
    switch (D) {
#define SBQA_ECB(D_)                                                                                                 \
    case D_: {                                                                                                       \
        const void *fn = reinterpret_cast<const void *>(&k_csr_energy_colblock<D_, FUSE>);                           \
        hipError_t e = ensure_dyn_lds(fn, lds);                                                                      \
        if (e != hipSuccess) return e;                                                                               \
        hipLaunchKernelGGL((k_csr_energy_colblock<D_, FUSE>), grid, block, lds, st, N, ld, nrb, rpb, RS, rcol, rval, \
                           rh, x, sbits, E, f);                                                                      \
        break;                                                                                                       \
    }
        SBQA_ECB(4) SBQA_ECB(6) SBQA_ECB(8) SBQA_ECB(12) SBQA_ECB(16)
#undef SBQA_ECB
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_csr_energy_colblock(int N, int ld, int C, int D, int nrb, int rpb, const int32_t *rcol,
                                      const double *rval, const double *rh, const float *x,
                                      const uint8_t *sbits, double *E, hipStream_t st) {
    return colblock_launch<false>(N, ld, C, D, nrb, rpb, rcol, rval, rh, x, sbits, E, ReadoutFuse{}, st);
}

hipError_t launch_csr_readout_colblock(int N, int ld, int C, int D, int nrb, int rpb, const int32_t *rcol,
                                       const double *rval, const double *rh, const float *x,
                                       const uint8_t *sbits, double *E, const ReadoutFuse &f, hipStream_t st) {
    return colblock_launch<true>(N, ld, C, D, nrb, rpb, rcol, rval, rh, x, sbits, E, f, st);
}

hipError_t launch_csr_energy_spins(int N, int count, const int32_t *row_ptr, const int32_t *col, const double *val,
                                   const Tri3 &t3, const double *h, const int8_t *spins, double *E, hipStream_t st) {
    hipLaunchKernelGGL(k_csr_energy_spins, dim3(count), dim3(256), 0, st, N, row_ptr, col, val, t3, h, spins, E);
    return hipGetLastError();
}

hipError_t launch_energy_fields(int N, int Np, int C, const float *x, const float *phi, const double *h, double *E,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_energy_fields, dim3(C), dim3(256), 0, st, N, Np, x, phi, h, E);
    return hipGetLastError();
}

hipError_t launch_best_update(int N, int R, int runs, int order, int ld, const float *x, const double *E,
                              double *best_E, int64_t *best_step, int8_t *best_spins, int64_t step, bool reset,
                              int *sel, hipStream_t st) {
    if (N > BEST_SPLIT_N && sel) {
        hipLaunchKernelGGL(k_best_select, dim3(runs), dim3(64), 0, st, R, E, best_E, best_step, sel, step,
                           reset ? 1 : 0);
        const int chunks = std::min(1024, (N + 256 * 8 - 1) / (256 * 8));
        hipLaunchKernelGGL(k_best_copy, dim3(chunks, runs), dim3(256), 0, st, N, R, order, ld, x, sel, best_spins);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_best_update, dim3(runs), dim3(1024), 0, st, N, R, order, ld, x, E, best_E, best_step,
                       best_spins, step, reset ? 1 : 0);
    return hipGetLastError();
}

}  // namespace sbqa
