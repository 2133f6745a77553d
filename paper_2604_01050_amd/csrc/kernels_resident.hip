// Register-resident CSR SBQA loop for gfx950: many steps of Eqs. 6-7 per
// launch (see the description below).
#include "csr_common.h"

#include <type_traits>

namespace sbqa {
namespace {

using namespace csr;

// ---------------------------------------------------------------------------
// Register-resident CSR loop: many steps per launch.
//
// One workgroup of NT threads (512, or 1024 from 2048 padded rows: the same
// rows in more waves hide more latency, 3-4% per step) owns RES_COLS consecutive replica
// columns of one run (R a multiple of RES_COLS) for all N spins. Its x and y
// and the fields h stay in registers for the whole launch; its operand f(X)
// for every spin (as binary16: -1, 0 and +1 are exact, and the coupling sum
// reads it with mixed-precision FMAs, no conversions) and its padded CSR
// weights stay in LDS; column indices stay in registers. The
// coupling sum of a column only needs that column's operand, so the only data
// that crosses workgroups is the ring coupling at the edges of the column
// block: after each step a workgroup publishes its first and last column and
// reads the neighbouring columns of the two workgroups next to it in the ring
// (coherent agent-scope accesses and per-workgroup step counters,
// double-buffered by step parity). Every wait is bounded: on timeout the error word is set and
// every later wait ends at once, so the grid always drains. The host launches
// the loop only when every workgroup fits on the device at once (occupancy
// times CUs); there is no grid-wide barrier, so an ordinary launch suffices.
// The state is stored column-block-major (ORDER_COLBLOCK8): the 8 columns of
// a workgroup for all rows are one contiguous run, so its starting loads and
// final stores are whole-line sequential accesses. The operand is not kept in
// memory between launches: each launch builds it from the starting x with the
// same f as the host-side operand rebuild.
// ---------------------------------------------------------------------------
constexpr int RES_COLS = 8;
constexpr int RES_MAX_ROWS = 4096;   // padded rows: a power of two from 512 to this
constexpr int RES_SPIN_LIMIT = 1 << 22;

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// The next step's operand is held as e4m3 bytes between the update and the
// barrier (2 registers per row instead of 4) and widened to binary16 when it
// is written to LDS; -1, 0 and +1 are exact in both formats.
__device__ __forceinline__ uint2 pack_e4m3(const float (&f)[RES_COLS]) {
    // the first conversion of each pair writes the low half of a register
    // whose previous contents (here an input that dies) are overwritten by
    // the second one
    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(f[0], f[1], __builtin_bit_cast(int, f[0]), false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(f[2], f[3], lo, true);
    int hi = __builtin_amdgcn_cvt_pk_fp8_f32(f[4], f[5], __builtin_bit_cast(int, f[4]), false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(f[6], f[7], hi, true);
    return make_uint2((uint32_t)lo, (uint32_t)hi);
}
__device__ __forceinline__ half8 e4m3_to_half(uint2 v) {
    const half2v a = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(v.x, 1.0f, false);
    const half2v b = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(v.x, 1.0f, true);
    const half2v c = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(v.y, 1.0f, false);
    const half2v d = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(v.y, 1.0f, true);
    half8 r;
    r[0] = a[0]; r[1] = a[1]; r[2] = b[0]; r[3] = b[1];
    r[4] = c[0]; r[5] = c[1]; r[6] = d[0]; r[7] = d[1];
    return r;
}

// Edge columns cross workgroups (possibly on different XCDs) through
// agent-scope atomic stores and loads: these are performed coherently for the
// whole device without writing back or invalidating the L2 caches. A producer
// waits for its stores to complete before its step counter is raised; a
// consumer reads the data only after it has seen the counter, so the data read
// is the data written for that step.
__device__ __forceinline__ void publish(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float fetch(const float *p) {
    return __hip_atomic_load(const_cast<float *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait of thread 0 until both ring-neighbour counters reach target; on
// timeout the error word is set and every later wait returns at once, so the
// grid always drains.
__device__ __forceinline__ void wait_neighbours(const int *cnt, int wl, int wr, int target, int *err) {
    int spins = 0;
    for (;;) {
        const int fl = __hip_atomic_load(const_cast<int *>(cnt) + wl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int fr = __hip_atomic_load(const_cast<int *>(cnt) + wr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fl >= target && fr >= target) break;
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (++spins > RES_SPIN_LIMIT) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

template <int RPT, int D, int NT>
__global__ __launch_bounds__(NT) void k_csr_resident(ResidentArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    // Rows are padded to NR = RPT*NT (zero rows: no field, no
    // couplings, zero state, so they stay zero); thread t owns rows
    // r = t + q*NT. LDS: binary16 operand of the own columns for
    // every row, then the weights laid out per thread so every thread
    // addresses them from one base with constant offsets.
    constexpr int NR = RPT * NT;
    half8 *op = reinterpret_cast<half8 *>(smem);                                            // [NR]
    float *wv = reinterpret_cast<float *>(smem + (size_t)NR * 16);                         // [RPT*D][T]
    const int t = threadIdx.x, w = blockIdx.x;
    const int P = a.R / RES_COLS;
    const int c0 = w * RES_COLS;
    const int run = c0 / a.R, part = (c0 - run * a.R) / RES_COLS;
    const int wl = run * P + (part + P - 1) % P, wr = run * P + (part + 1) % P;

    // the prologue issues all of its global loads (weights, state, column
    // indices of every row) before it waits for any of them: one memory
    // round trip instead of one per row and kind
    float wtmp[RPT][D];
    int32_t ctmp[RPT][D];
    float xs[RPT][RES_COLS], ys[RPT][RES_COLS];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = t + q * NT;
#pragma unroll
        for (int p = 0; p < D; ++p) wtmp[q][p] = a.valpad[(int64_t)p * NR + r];
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = t + q * NT;
        const float *xrow = a.x + ((int64_t)w * NR + r) * RES_COLS;
        const float *yrow = a.y + ((int64_t)w * NR + r) * RES_COLS;
        const float4 x0 = *reinterpret_cast<const float4 *>(xrow);
        const float4 x1 = *reinterpret_cast<const float4 *>(xrow + 4);
        const float4 y0 = *reinterpret_cast<const float4 *>(yrow);
        const float4 y1 = *reinterpret_cast<const float4 *>(yrow + 4);
        xs[q][0] = x0.x; xs[q][1] = x0.y; xs[q][2] = x0.z; xs[q][3] = x0.w;
        xs[q][4] = x1.x; xs[q][5] = x1.y; xs[q][6] = x1.z; xs[q][7] = x1.w;
        ys[q][0] = y0.x; ys[q][1] = y0.y; ys[q][2] = y0.z; ys[q][3] = y0.w;
        ys[q][4] = y1.x; ys[q][5] = y1.y; ys[q][6] = y1.z; ys[q][7] = y1.w;
#pragma unroll
        for (int p = 0; p < D; ++p) ctmp[q][p] = a.colpad[(int64_t)r * D + p];
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int p = 0; p < D; ++p) wv[(q * D + p) * NT + t] = wtmp[q][p];

    uint32_t cpk[RPT][(D + 1) / 2];
    // exchange buffer of parity b, block v, edge e (0: first column, 1: last),
    // indexed by row (consecutive lanes, consecutive addresses)
    auto slot = [&](int b, int v, int e) { return a.xpub + (((int64_t)b * a.nwg + v) * 2 + e) * NR; };
    {
        float *pf = slot(a.n0 & 1, w, 0), *pl = slot(a.n0 & 1, w, 1);
        const float d0 = a.delta[a.n0];   // the operand of step n0 is f(x) at Delta_n0
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = t + q * NT;
            half8 f0;
#pragma unroll
            for (int c = 0; c < RES_COLS; ++c) f0[c] = (_Float16)f_value(a.fmode, xs[q][c], d0);
            op[r] = f0;
#pragma unroll
            for (int p = 0; p < D; p += 2) {
                // LDS byte offsets of the neighbours' operand rows (< 2^16)
                const uint32_t j0 = (uint32_t)ctmp[q][p] * (uint32_t)sizeof(half8);
                const uint32_t j1 = (p + 1 < D) ? (uint32_t)ctmp[q][p + 1] * (uint32_t)sizeof(half8) : 0u;
                cpk[q][p / 2] = j0 | (j1 << 16);
            }
            publish(pf + r, xs[q][0]);                   // edges of the starting state
            publish(pl + r, xs[q][RES_COLS - 1]);
        }
    }
    // one round on the launch counters: every block's starting edges are out
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (t == 0) {
        __hip_atomic_store(a.epoch_cnt + w, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_neighbours(a.epoch_cnt, wl, wr, a.epoch, a.err);
    }
    __syncthreads();

    float kA = a.coefA[a.n0], dn = a.delta[a.n0 + 1], jpr = a.jp[(int64_t)run * a.S + a.n0];
    // one step; the launch's last one (LAST) is a separate copy that stores
    // each row's final state as soon as the row is updated, so that the
    // stores drain while the other rows compute, and skips the hand-over to
    // a next step (with the stores in the loop itself the loop needed 27 more
    // registers and ran 2% slower)
    auto step = [&](int s, auto last_c) __attribute__((always_inline)) {
        constexpr bool LAST = decltype(last_c)::value;
        // compiler-only barriers: the loop-invariant LDS weights are re-read
        // every step instead of being pinned in registers, and the packed
        // neighbour offsets are unpacked every step instead of being kept
        // unpacked (twice the registers)
        asm volatile("" ::: "memory");
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int i = 0; i < (D + 1) / 2; ++i) asm volatile("" : "+v"(cpk[q][i]));
        const int n = a.n0 + s;
        const float d = (a.fmode == 1) ? 0.0f : dn;
        const float kA_n = kA, jp_n = jpr;
        if (!LAST) {  // the next step's scalars load while this step runs
            kA = a.coefA[n + 1];
            dn = a.delta[n + 2];
            jpr = a.jp[(int64_t)run * a.S + n + 1];
        }
        const float *publ = slot(n & 1, wl, 1);   // last column of the left block
        const float *pubr = slot(n & 1, wr, 0);   // first column of the right block
        // this step's edges go out row by row as soon as a row is updated: the
        // parity-(n+1) slots were last read by the neighbours in step n-1,
        // which they had finished when this block passed its last wait
        float *pf = slot((n + 1) & 1, w, 0), *pl = slot((n + 1) & 1, w, 1);
        uint2 fnew[RPT];
        // one row ahead: the fields h (re-read every step, cache-resident)
        // and the ring-neighbour edge values (coherent loads, long latency)
        float hnext = a.h[t], lnext = fetch(publ + t), rnext = fetch(pubr + t);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int r = t + q * NT;
            asm volatile("" : "+v"(r));
            const float hq = hnext, lq = lnext, rq = rnext;
            if (q + 1 < RPT) {
                hnext = a.h[r + NT];
                lnext = fetch(publ + r + NT);
                rnext = fetch(pubr + r + NT);
            }
            float acc[RES_COLS];
#pragma unroll
            for (int c = 0; c < RES_COLS; ++c) acc[c] = 0.f;
#pragma unroll
            for (int p = 0; p < D; ++p) {
                const uint32_t jo = (cpk[q][p / 2] >> (16 * (p & 1))) & 0xFFFFu;
                const half8 f = *reinterpret_cast<const half8 *>(smem + jo);
                const float wgt = wv[(q * D + p) * NT + t];
                // binary16 -1, 0, +1 widen exactly: the same bits as a float32 operand
#pragma unroll
                for (int c = 0; c < RES_COLS; ++c) acc[c] = __builtin_fmaf(wgt, (float)f[c], acc[c]);
            }
            const float br = rq;
            // columns left to right, in place: the left ring term reads the
            // step-n value of column c-1 kept in prev, the right one the
            // not yet updated column c+1
            float prev = lq;
            float fv[RES_COLS];
#pragma unroll
            for (int c = 0; c < RES_COLS; ++c) {
                const float xr = c == RES_COLS - 1 ? br : xs[q][c + 1];
                float xn, yn, sg;
                update_elem(xs[q][c], ys[q][c], acc[c], hq, prev, xr, jp_n, kA_n, a.kB, a.dt, a.kD, xn, yn, sg);
                // f of Eq. 8 (d = 0 for sign): the value ternary_byte gives
                fv[c] = fabsf(xn) > d ? sg : 0.0f;
                prev = xs[q][c];
                xs[q][c] = xn;
                ys[q][c] = yn;
            }
            // materialise y here: otherwise the wall's selects are sunk to the
            // next step and their condition masks pile up in scalar registers
#pragma unroll
            for (int c = 0; c < RES_COLS; ++c) asm volatile("" : "+v"(ys[q][c]));
            if constexpr (LAST) {
                // the final state of the row, and one byte of sign bits (bit
                // c: column c negative) for the readout energies
                float *xrow = a.x + ((int64_t)w * NR + r) * RES_COLS;
                float *yrow = a.y + ((int64_t)w * NR + r) * RES_COLS;
                *reinterpret_cast<float4 *>(xrow) = make_float4(xs[q][0], xs[q][1], xs[q][2], xs[q][3]);
                *reinterpret_cast<float4 *>(xrow + 4) = make_float4(xs[q][4], xs[q][5], xs[q][6], xs[q][7]);
                *reinterpret_cast<float4 *>(yrow) = make_float4(ys[q][0], ys[q][1], ys[q][2], ys[q][3]);
                *reinterpret_cast<float4 *>(yrow + 4) = make_float4(ys[q][4], ys[q][5], ys[q][6], ys[q][7]);
                uint32_t sb = 0;
#pragma unroll
                for (int c = 0; c < RES_COLS; ++c) sb |= (xs[q][c] < 0.0f ? 1u : 0u) << c;
                a.sbits[(int64_t)w * NR + r] = (uint8_t)sb;
            } else {
                fnew[q] = pack_e4m3(fv);
                publish(pf + r, xs[q][0]);
                publish(pl + r, xs[q][RES_COLS - 1]);
            }
            // keep rows apart in the schedule: hoisting every row's gathers
            // ahead raises the register demand past two waves per SIMD
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (LAST) return;
        __syncthreads();  // every wave is done reading the step-n operand
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int r = t + q * NT;
            asm volatile("" : "+v"(r));
            op[r] = e4m3_to_half(fnew[q]);
        }
        __builtin_amdgcn_s_waitcnt(0);  // this wave's edge stores have completed
        __syncthreads();
        if (t == 0) {
            __hip_atomic_store(a.flags + w, n + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            wait_neighbours(a.flags, wl, wr, n + 1, a.err);
        }
        __syncthreads();
    };
    for (int s = 0; s + 1 < a.K; ++s) step(s, std::false_type{});
    step(a.K - 1, std::true_type{});
}

}  // namespace

int resident_degree(int maxdeg) {
    const int opts[] = {4, 6, 8, 12, 16};
    for (int d : opts)
        if (maxdeg <= d) return d;
    return -1;
}

// rows of the resident kernel: N padded to a power of two, at least 512
int resident_rows(int N) {
    if (N < 1 || N > RES_MAX_ROWS) return -1;
    int nr = 512;
    while (nr < N) nr *= 2;
    return nr;
}

size_t resident_lds_bytes(int N, int D) {
    const int rows = resident_rows(N);
    return rows < 0 ? 0 : (size_t)rows * (16 + 4 * D);
}

// threads per workgroup: 1024 from 2048 rows (measured per step, 6-regular,
// 2048 columns: 4096 rows 6.96 against 7.22 us, 2048 rows 4.12 against 4.31;
// at 1024 rows 512 threads are 1-2% faster)
int resident_threads(int N) {
    const int rows = resident_rows(N);
    return rows < 0 ? -1 : rows >= 2048 ? 1024 : 512;
}

// rows per thread (1, 2 or 4), or -1 when N is too large
int resident_rpt(int N) {
    const int rows = resident_rows(N);
    return rows < 0 ? -1 : rows / resident_threads(N);
}

int resident_cols() { return RES_COLS; }

// The instances that are built: 512 threads with 1 or 2 rows each, 1024
// threads with 2 or 4 rows each (4 only up to degree 6: the register budget
// of four waves per SIMD).
template <int RPT, int NT>
constexpr bool res_built(int D) {
    return (NT == 512 && (RPT == 1 || RPT == 2)) || (NT == 1024 && (RPT == 2 || (RPT == 4 && D <= 6)));
}

template <class F>
static hipError_t with_resident(int RPT, int D, int NT, F &&f) {
    auto by_d = [&](auto rpt_c, auto nt_c) -> hipError_t {
        constexpr int R_ = decltype(rpt_c)::value, T_ = decltype(nt_c)::value;
        switch (D) {
            case 4: return f(&k_csr_resident<R_, 4, T_>, T_);
            case 6: return f(&k_csr_resident<R_, 6, T_>, T_);
            case 8: if constexpr (res_built<R_, T_>(8)) return f(&k_csr_resident<R_, 8, T_>, T_); else break;
            case 12: if constexpr (res_built<R_, T_>(12)) return f(&k_csr_resident<R_, 12, T_>, T_); else break;
            case 16: if constexpr (res_built<R_, T_>(16)) return f(&k_csr_resident<R_, 16, T_>, T_); else break;
            default: break;
        }
        return hipErrorInvalidValue;
    };
    using I = std::integral_constant<int, 1>;
    using II = std::integral_constant<int, 2>;
    using IV = std::integral_constant<int, 4>;
    using T5 = std::integral_constant<int, 512>;
    using T10 = std::integral_constant<int, 1024>;
    if (NT == 512 && RPT == 1) return by_d(I{}, T5{});
    if (NT == 512 && RPT == 2) return by_d(II{}, T5{});
    if (NT == 1024 && RPT == 2) return by_d(II{}, T10{});
    if (NT == 1024 && RPT == 4) return by_d(IV{}, T10{});
    return hipErrorInvalidValue;
}

hipError_t launch_csr_resident(const ResidentArgs &a, int D, hipStream_t st) {
    const int rpt = resident_rpt(a.N), nt = resident_threads(a.N);
    if (a.R % RES_COLS || rpt < 0 || a.N > 65535) return hipErrorInvalidValue;
    const size_t lds = resident_lds_bytes(a.N, D);
    return with_resident(rpt, D, nt, [&](auto kern, int threads) -> hipError_t {
        const void *fn = reinterpret_cast<const void *>(kern);
        hipError_t e = ensure_dyn_lds(fn, lds);
        if (e != hipSuccess) return e;
        ResidentArgs arg = a;
        void *args[] = {&arg};
        return hipLaunchKernel(fn, dim3(a.nwg), dim3(threads), args, (unsigned)lds, st);
    });
}

hipError_t resident_max_blocks(int D, int N, int *blocks_per_cu) {
    const int rpt = resident_rpt(N), nt = resident_threads(N);
    const size_t lds = resident_lds_bytes(N, D);
    return with_resident(rpt, D, nt, [&](auto kern, int threads) -> hipError_t {
        const void *fn = reinterpret_cast<const void *>(kern);
        hipError_t e = ensure_dyn_lds(fn, lds);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, threads, lds);
    });
}

}  // namespace sbqa
