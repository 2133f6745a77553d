// Resident loop for small dense instances (gfx950): one workgroup per run;
// each thread keeps one row of J (float32) in registers for the whole launch
// and owns that spin in some of the run's replicas, whose positions and
// operand sit in LDS (every lane of a wave reads the same operand row, a
// broadcast) and whose velocities stay in registers; the loop advances K
// steps of Eqs. 6-7 per launch, so a small all-to-all instance costs one
// launch per K steps instead of one per step. Fields are summed in a fixed
// order over j (four interleaved partial sums), so integer couplings with a
// ternary or sign operand give exactly the fields of the MFMA path. For J in
// {-1, 0, +1} with such an operand a second form (k_dense_small_bits, below)
// replaces the FMAs by bit counts over masks of J and of the operand.
#include "sbqa_internal.h"

#include <type_traits>

namespace sbqa {
namespace {

constexpr int SM_THREADS = 512;   // two waves per SIMD
// replica-spin elements per thread: thread t keeps row i = t % N of J in
// registers and owns replicas t / N + m * (SM_THREADS / N); the largest m
// count over N <= SMALL_MAX_N and R * N <= SMALL_MAX_ELEMS is 10 (N = 104)
constexpr int SM_EPT = 10;

// operand row length in LDS: N rounded up to the kernel's 32, 64 or 128
__host__ __device__ constexpr int small_rows(int N) { return N <= 32 ? 32 : N <= 64 ? 64 : 128; }

__device__ __forceinline__ float f_small(int fmode, float x, float delta) {
    if (fmode == 2) return x;                       // bSB
    const float d = (fmode == 1) ? 0.0f : delta;    // dSB: sign(0) = 0
    if (fabsf(x) <= d) return 0.0f;
    return x > 0.0f ? 1.0f : -1.0f;
}

#pragma clang fp contract(off)
// Eqs. 6-7 for one replica-spin element: the kick with the coupling sum phi,
// the fields, the ring neighbours' positions xl, xr and the pumping term,
// then the drift and the wall of Eq. 3; returns the new position, y updated
// in place
__device__ __forceinline__ float small_update(float x, float xl, float xr, float phi, float h, float &y, float kA,
                                              float jpr, const SmallArgs &a) {
    const float force = (-kA * x + a.kB * (phi + h)) + jpr * (xl + xr);
    float yn = y + a.dt * force;
    float xv = x + a.kD * yn;
    if (fabsf(xv) > 1.0f) {
        xv = xv > 0.0f ? 1.0f : -1.0f;
        yn = 0.0f;
    }
    y = yn;
    return xv;
}

// NMAX: N rounded up to 32, 64 or 128 (J row registers, operand rows in LDS,
// both zero past N, so the coupling sum runs over NMAX terms without bounds);
// M: replicas per thread, ceil(R / (SM_THREADS / N)) rounded up to 1, 2, 4 or
// SM_EPT
template <int NMAX, int M>
__global__ __launch_bounds__(SM_THREADS) void k_dense_small(const SmallArgs a) {
    extern __shared__ __align__(16) float sm[];
    const int N = a.N, R = a.R, NS = NMAX;
    // two buffers, each [R][NS] positions of this run then [R][NS] operand
    // f(x) (zero past N): step n reads one and writes the other, so one
    // barrier per step orders both its reads and the next step's
    float *const buf0 = sm, *const buf1 = sm + 2 * R * NS;
    const int run = blockIdx.x, tid = threadIdx.x;
    const int G = SM_THREADS / N, i = tid % N, g = tid / N;
    const bool active = g < G;
    // row i of J, zero past N: the padding terms add +0 to sums that start
    // at +0 and so never hold -0
    float jr[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) jr[j] = (active && j < N) ? a.J[(int64_t)i * N + j] : 0.0f;
    for (int e = tid; e < R * NS; e += SM_THREADS) {
        buf0[R * NS + e] = 0.0f;
        buf1[R * NS + e] = 0.0f;
    }
    __syncthreads();
    // this thread's replicas k = g + m * G
    float yv[M], hv[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = g + m * G;
        if (active && k < R) {
            const int64_t o = (int64_t)(run * R + k) * a.Np + i;
            const float x = a.x[o];
            buf0[k * NS + i] = x;
            buf0[R * NS + k * NS + i] = f_small(a.fmode, x, a.delta[a.n0]);
            yv[m] = a.y[o];
            hv[m] = a.h[i];
        }
    }
    __syncthreads();

    // the step's scalars are loaded one step ahead (their loads drain while
    // the previous step runs instead of stalling the update)
    float kA_next = a.coefA[a.n0], dnext_next = a.delta[a.n0 + 1], jpr_next = a.jp[(int64_t)run * a.S + a.n0];
    for (int n = a.n0; n < a.n0 + a.K; ++n) {
        const float kA = kA_next, dnext = dnext_next, jpr = jpr_next;
        if (n + 1 < a.n0 + a.K) {
            kA_next = a.coefA[n + 1];
            dnext_next = a.delta[n + 2];
            jpr_next = a.jp[(int64_t)run * a.S + n + 1];
        }
        const bool odd = (n - a.n0) & 1;
        const float *xs = odd ? buf1 : buf0, *fs = xs + R * NS;
        float *xo = odd ? buf0 : buf1, *fo = xo + R * NS;
        float xn[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = g + m * G;
            if (!active || k >= R) continue;
            const float4 *frow = reinterpret_cast<const float4 *>(fs + k * NS);
            // four interleaved partial sums over j = 4m + u < NMAX, then
            // (s0 + s1) + (s2 + s3): a fixed order with four independent FMA
            // chains (the terms past N are +0 * +0 on sums that start at +0)
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
            for (int j = 0; j < NMAX; j += 4) {
                const float4 f = frow[j / 4];
                s0 = fmaf(jr[j], f.x, s0);
                s1 = fmaf(jr[j + 1], f.y, s1);
                s2 = fmaf(jr[j + 2], f.z, s2);
                s3 = fmaf(jr[j + 3], f.w, s3);
            }
            const float phi = (s0 + s1) + (s2 + s3);
            const int kl = (k == 0) ? R - 1 : k - 1, kr = (k == R - 1) ? 0 : k + 1;
            xn[m] = small_update(xs[k * NS + i], xs[kl * NS + i], xs[kr * NS + i], phi, hv[m], yv[m], kA, jpr, a);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = g + m * G;
            if (!active || k >= R) continue;
            xo[k * NS + i] = xn[m];
            fo[k * NS + i] = f_small(a.fmode, xn[m], dnext);
        }
        __syncthreads();   // step n + 1 reads what step n wrote; step n's reads are done
    }
    const float *xs = (a.K & 1) ? buf1 : buf0;   // the buffer the last step wrote
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = g + m * G;
        if (!active || k >= R) continue;
        const int64_t o = (int64_t)(run * R + k) * a.Np + i;
        a.x[o] = xs[k * NS + i];
        a.y[o] = yv[m];
    }
}
// The same loop for J in {-1, 0, +1} with a ternary or sign operand, laid
// out by NMAX = N rounded up to 32, 64 or 128 (lane i % NMAX holds spin i;
// lanes past N idle), so that the spins of one replica sit in one half-wave
// (NMAX = 32), one wave (64) or two waves (128), lane order = spin order.
// Each lane keeps row i of J as bit masks (nonzero, negative) and the
// operand of its replica as masks of the same form, taken with wave ballots
// right after the update: a wave's own 64 (or 32) spins stay in registers,
// and with two waves per replica each wave passes its half to the other
// through LDS, double-buffered with the positions. The coupling sum is then
// an exact integer count: the terms with both factors nonzero, minus twice
// those whose product is negative,
//   phi_i = popc(nzJ_i & nzF) - 2 popc(nzJ_i & nzF & (negJ_i ^ negF)),
// the value the float32 sum of the other kernel reaches exactly (|phi| <= N),
// so both kernels give the same bits. Positions of the ring neighbours (other
// waves) go through LDS too, one barrier per step.
// (FULL: N = NMAX, every lane holds a spin)
template <int NMAX, int M, bool FULL>
__global__ __launch_bounds__(SM_THREADS) void k_dense_small_bits(const SmallArgs a) {
    static_assert(NMAX == 32 || NMAX == 64 || NMAX == 128, "a replica's spins in a half-wave, a wave or two");
    constexpr bool TWO = NMAX == 128;               // two waves per replica
    constexpr int JW = NMAX < 64 ? NMAX : 64;       // spins per mask word
    extern __shared__ __align__(16) float sm[];
    const int R = a.R, NS = NMAX;
    float *const buf0 = sm, *const buf1 = sm + R * NS;   // [R][NS] positions each
    // two waves per replica: [parity][R][half][nonzero, negative] masks
    uint64_t *const mk = reinterpret_cast<uint64_t *>(sm + 2 * R * NS);
    const int run = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    constexpr int G = SM_THREADS / NMAX;
    const int N = a.N, i = tid % NMAX, g = tid / NMAX;
    const bool row = FULL || i < N;
    // this lane's bits in its wave's ballot: lanes [32 hw, 32 hw + 32) for
    // NMAX = 32, all 64 otherwise; hh: the half of the replica this wave holds
    const int hw = NMAX == 32 ? lane >> 5 : 0;
    const int hh = TWO ? (tid >> 6) & 1 : 0;
    auto own = [&](uint64_t b) -> uint64_t { return NMAX == 32 ? (b >> (32 * hw)) & 0xFFFFFFFFull : b; };
    // row i of J over the wave's own spins (jnz, jneg) and over the other
    // wave's (onz, oneg: two waves per replica only); zero past N and for
    // idle lanes
    uint64_t jnz = 0, jneg = 0, onz = 0, oneg = 0;
#pragma unroll
    for (int j = 0; j < JW; ++j) {
        const int cm = hh * 64 + j, co = (1 - hh) * 64 + j;
        const float v = (row && cm < N) ? a.J[(int64_t)i * N + cm] : 0.0f;
        jnz |= (uint64_t)(v != 0.0f) << j;
        jneg |= (uint64_t)(v < 0.0f) << j;
        if constexpr (TWO) {
            const float u = (row && co < N) ? a.J[(int64_t)i * N + co] : 0.0f;
            onz |= (uint64_t)(u != 0.0f) << j;
            oneg |= (uint64_t)(u < 0.0f) << j;
        }
    }
    // this thread's replicas k = g + m * G (the same k across a wave or
    // half-wave, so every ballot below covers whole replicas or halves)
    float yv[M], hv[M];
    uint64_t fnz[M], fneg[M];
    // the wave's operand masks of replica k for the readers of parity b
    auto pass = [&](int b, int k, uint64_t nz, uint64_t ng) {
        if (TWO && lane == 0 && k < R) {
            mk[((b * R + k) * 2 + hh) * 2] = nz;
            mk[((b * R + k) * 2 + hh) * 2 + 1] = ng;
        }
    };
    // the lane's own positions stay in registers too (xc); with one wave or
    // half-wave per replica the operand masks are taken at the start of each
    // step, after the barrier, where they overlap the neighbours' LDS reads
    float xc[M];
    float dcur = a.fmode == 1 ? 0.0f : a.delta[a.n0];   // the operand's Delta
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = g + m * G;
        const bool valid = row && k < R;
        float x = 0.0f;
        if (valid) {
            const int64_t o = (int64_t)(run * R + k) * a.Np + i;
            x = a.x[o];
            buf0[k * NS + i] = x;
            yv[m] = a.y[o];
            hv[m] = a.h[i];
        }
        xc[m] = x;
        if constexpr (TWO) {
            fnz[m] = __ballot(valid && !(fabsf(x) <= dcur));
            fneg[m] = __ballot(valid && !(fabsf(x) <= dcur) && !(x > 0.0f));
            pass(0, k, fnz[m], fneg[m]);
        }
    }
    __syncthreads();

    float kA_next = a.coefA[a.n0], dnext_next = a.delta[a.n0 + 1], jpr_next = a.jp[(int64_t)run * a.S + a.n0];
    for (int n = a.n0; n < a.n0 + a.K; ++n) {
        const float kA = kA_next, dnext = dnext_next, jpr = jpr_next;
        if (n + 1 < a.n0 + a.K) {
            kA_next = a.coefA[n + 1];
            dnext_next = a.delta[n + 2];
            jpr_next = a.jp[(int64_t)run * a.S + n + 1];
        }
        const float d = a.fmode == 1 ? 0.0f : dnext;
        const int odd = (n - a.n0) & 1;
        const float *xs = odd ? buf1 : buf0;
        float *xo = odd ? buf0 : buf1;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = g + m * G;
            const bool valid = row && k < R;
            if constexpr (!TWO) {
                // f of Eq. 8 (d = 0 for sign), with the comparisons of f_small
                fnz[m] = own(__ballot(valid && !(fabsf(xc[m]) <= dcur)));
                fneg[m] = own(__ballot(valid && !(fabsf(xc[m]) <= dcur) && !(xc[m] > 0.0f)));
            }
            float xv = 0.0f;
            if (valid) {
                const uint64_t both = jnz & fnz[m], minus = both & (jneg ^ fneg[m]);
                // (the counts are unsigned: the difference is formed as int)
                int cnt = (int)__popcll(both) - 2 * (int)__popcll(minus);
                if constexpr (TWO) {
                    const uint64_t *om = mk + ((odd * R + k) * 2 + 1 - hh) * 2;
                    const uint64_t b2 = onz & om[0], m2 = b2 & (oneg ^ om[1]);
                    cnt += (int)__popcll(b2) - 2 * (int)__popcll(m2);
                }
                const float phi = (float)cnt;
                const int kl = (k == 0) ? R - 1 : k - 1, kr = (k == R - 1) ? 0 : k + 1;
                xv = small_update(xc[m], xs[kl * NS + i], xs[kr * NS + i], phi, hv[m], yv[m], kA, jpr, a);
                xo[k * NS + i] = xv;
            }
            xc[m] = xv;
            if constexpr (TWO) {
                // the masks of the next step's operand (Delta d) for both
                // waves of the replica, before the barrier
                fnz[m] = __ballot(valid && !(fabsf(xv) <= d));
                fneg[m] = __ballot(valid && !(fabsf(xv) <= d) && !(xv > 0.0f));
                pass(1 - odd, k, fnz[m], fneg[m]);
            }
        }
        dcur = d;
        __syncthreads();   // step n + 1 reads what step n wrote; step n's reads are done
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int k = g + m * G;
        if (!row || k >= R) continue;
        const int64_t o = (int64_t)(run * R + k) * a.Np + i;
        a.x[o] = xc[m];
        a.y[o] = yv[m];
    }
}
#pragma clang fp contract(on)

}  // namespace

size_t small_lds_bytes(int N, int R) { return sizeof(float) * 4 * (size_t)R * small_rows(N); }

hipError_t launch_dense_small(const SmallArgs &a, int runs, hipStream_t st) {
    if (a.N < 1 || a.N > SMALL_MAX_N || a.R < 1 || a.R * a.N > SMALL_MAX_ELEMS || a.K < 1 || a.n0 < 0 ||
        a.n0 + a.K > a.S)
        return hipErrorInvalidValue;
    // every replica of the run has a thread group: R <= SM_EPT * (SM_THREADS / N)
    if (a.R > SM_EPT * (SM_THREADS / a.N)) return hipErrorInvalidValue;
    const size_t lds = small_lds_bytes(a.N, a.R);
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = ensure_dyn_lds(reinterpret_cast<const void *>(kern), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(runs), dim3(SM_THREADS), lds, st, a);
        return hipGetLastError();
    };
    const int G = SM_THREADS / a.N, m = (a.R + G - 1) / G;
    // the bit-mask loop: groups of NMAX = 32, 64 or 128 lanes per replica, at
    // most 8 replicas per thread (a larger R keeps the float32 loop)
    const int nb = small_rows(a.N), Gb = SM_THREADS / nb, mb = (a.R + Gb - 1) / Gb;
    if (a.jbits && a.fmode != 2 && mb <= 8) {
        auto by_mb = [&](auto nmax, auto full) -> hipError_t {
            constexpr int NM = decltype(nmax)::value;
            constexpr bool F = decltype(full)::value;
            if (mb <= 1) return go(&k_dense_small_bits<NM, 1, F>);
            if (mb <= 2) return go(&k_dense_small_bits<NM, 2, F>);
            if (mb <= 4) return go(&k_dense_small_bits<NM, 4, F>);
            return go(&k_dense_small_bits<NM, 8, F>);
        };
        auto by_full = [&](auto nmax) -> hipError_t {
            if (a.N == decltype(nmax)::value) return by_mb(nmax, std::true_type{});
            return by_mb(nmax, std::false_type{});
        };
        if (nb == 32) return by_full(std::integral_constant<int, 32>{});
        if (nb == 64) return by_full(std::integral_constant<int, 64>{});
        return by_full(std::integral_constant<int, 128>{});
    }
    auto by_m = [&](auto nmax) -> hipError_t {
        constexpr int NM = decltype(nmax)::value;
        if (m <= 1) return go(&k_dense_small<NM, 1>);
        if (m <= 2) return go(&k_dense_small<NM, 2>);
        if (m <= 4) return go(&k_dense_small<NM, 4>);
        return go(&k_dense_small<NM, SM_EPT>);
    };
    if (a.N <= 32) return by_m(std::integral_constant<int, 32>{});
    if (a.N <= 64) return by_m(std::integral_constant<int, 64>{});
    return by_m(std::integral_constant<int, 128>{});
}

}  // namespace sbqa
