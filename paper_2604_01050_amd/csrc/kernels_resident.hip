// Register-resident CSR SBQA loop for gfx950: many steps of Eqs. 6-7 per
// cooperative launch (see the description below).
#include "csr_common.h"

namespace sbqa {
namespace {

using namespace csr;

// ---------------------------------------------------------------------------
// Register-resident CSR loop: many steps per launch.
//
// One workgroup of RES_THREADS threads owns RES_COLS consecutive replica
// columns of one run (R a multiple of RES_COLS) for all N spins. Its x and y
// stay in registers for the whole launch; its operand f(X) for every spin and
// its padded CSR weights stay in LDS; column indices stay in registers. The
// coupling sum of a column only needs that column's operand, so the only data
// that crosses workgroups is the ring coupling at the edges of the column
// block: after each step a workgroup publishes its first and last column and
// reads the neighbouring columns of the two workgroups next to it in the ring
// (coherent agent-scope accesses and per-workgroup step counters,
// double-buffered by step parity). Every wait is bounded: on timeout the error word is set and
// every later wait ends at once, so the grid always drains. The launch is
// cooperative, so all workgroups are co-resident.
// ---------------------------------------------------------------------------
constexpr int RES_COLS = 8;
constexpr int RES_THREADS = 512;
constexpr int RES_MAX_RPT = 8;
constexpr int RES_SPIN_LIMIT = 1 << 22;

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

template <int RPT, int D>
__global__ __launch_bounds__(RES_THREADS) void k_csr_resident(ResidentArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    // Rows are padded to NR = RPT*RES_THREADS (zero rows: no field, no
    // couplings, zero state, so they stay zero). LDS: operand of the own
    // columns for every row, then the weights and fields laid out per thread
    // (row r = t + q*RES_THREADS) so every thread addresses them from one base
    // with constant offsets.
    constexpr int NR = RPT * RES_THREADS;
    uint2 *op = reinterpret_cast<uint2 *>(smem);                                            // [NR]
    float *wv = reinterpret_cast<float *>(smem + (size_t)NR * 8);                          // [RPT*D][T]
    float *hs = reinterpret_cast<float *>(smem + (size_t)NR * 8 + (size_t)RPT * D * RES_THREADS * 4);  // [RPT][T]
    const int t = threadIdx.x, w = blockIdx.x;
    const int P = a.R / RES_COLS;
    const int c0 = w * RES_COLS;
    const int run = c0 / a.R, part = (c0 - run * a.R) / RES_COLS;
    const int wl = run * P + (part + P - 1) % P, wr = run * P + (part + 1) % P;

#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        int r = t + q * RES_THREADS;
        asm volatile("" : "+v"(r));
        op[r] = *reinterpret_cast<const uint2 *>(a.g + (int64_t)r * a.Cs + c0);
        hs[q * RES_THREADS + t] = a.h[r];
#pragma unroll
        for (int p = 0; p < D; ++p) wv[(q * D + p) * RES_THREADS + t] = a.valpad[(int64_t)p * NR + r];
    }

    float xs[RPT][RES_COLS], ys[RPT][RES_COLS];
    uint32_t cpk[RPT][(D + 1) / 2];
    // exchange buffer of parity b, block v, edge e (0: first column, 1: last)
    auto slot = [&](int b, int v, int e) { return a.xpub + (((int64_t)b * a.nwg + v) * 2 + e) * NR; };
    {
        float *pf = slot(a.n0 & 1, w, 0), *pl = slot(a.n0 & 1, w, 1);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int r = t + q * RES_THREADS;
            asm volatile("" : "+v"(r));
            const float *xrow = a.x + (int64_t)r * a.Cs + c0;
            const float *yrow = a.y + (int64_t)r * a.Cs + c0;
            const float4 x0 = *reinterpret_cast<const float4 *>(xrow);
            const float4 x1 = *reinterpret_cast<const float4 *>(xrow + 4);
            const float4 y0 = *reinterpret_cast<const float4 *>(yrow);
            const float4 y1 = *reinterpret_cast<const float4 *>(yrow + 4);
            xs[q][0] = x0.x; xs[q][1] = x0.y; xs[q][2] = x0.z; xs[q][3] = x0.w;
            xs[q][4] = x1.x; xs[q][5] = x1.y; xs[q][6] = x1.z; xs[q][7] = x1.w;
            ys[q][0] = y0.x; ys[q][1] = y0.y; ys[q][2] = y0.z; ys[q][3] = y0.w;
            ys[q][4] = y1.x; ys[q][5] = y1.y; ys[q][6] = y1.z; ys[q][7] = y1.w;
#pragma unroll
            for (int p = 0; p < D; p += 2) {
                const uint32_t j0 = (uint32_t)a.colpad[(int64_t)r * D + p];
                const uint32_t j1 = (p + 1 < D) ? (uint32_t)a.colpad[(int64_t)r * D + p + 1] : 0u;
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
    for (int s = 0; s < a.K; ++s) {
        // compiler-only barrier: the loop-invariant LDS weights and fields are
        // re-read every step instead of being pinned in registers
        asm volatile("" ::: "memory");
        const int n = a.n0 + s;
        const float d = (a.fmode == 1) ? 0.0f : dn;
        const float kA_n = kA, jp_n = jpr;
        if (s + 1 < a.K) {  // the next step's scalars load while this step runs
            kA = a.coefA[n + 1];
            dn = a.delta[n + 2];
            jpr = a.jp[(int64_t)run * a.S + n + 1];
        }
        const float *publ = slot(n & 1, wl, 1);   // last column of the left block
        const float *pubr = slot(n & 1, wr, 0);   // first column of the right block
        uint2 fnew[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int r = t + q * RES_THREADS;
            asm volatile("" : "+v"(r));
            float acc[RES_COLS];
#pragma unroll
            for (int c = 0; c < RES_COLS; ++c) acc[c] = 0.f;
#pragma unroll
            for (int p = 0; p < D; ++p) {
                const uint32_t j = (cpk[q][p / 2] >> (16 * (p & 1))) & 0xFFFFu;
                const uint2 f8 = op[j];
                const float wgt = wv[(q * D + p) * RES_THREADS + t];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    acc[c] = __builtin_fmaf(wgt, (float)(int8_t)((f8.x >> (8 * c)) & 0xFF), acc[c]);
                    acc[c + 4] = __builtin_fmaf(wgt, (float)(int8_t)((f8.y >> (8 * c)) & 0xFF), acc[c + 4]);
                }
            }
            const float hv = hs[q * RES_THREADS + t];
            const float br = fetch(pubr + r);
            // columns left to right, in place: the left ring term reads the
            // step-n value of column c-1 kept in prev, the right one the
            // not yet updated column c+1
            uint32_t lo = 0, hi = 0;
            float prev = fetch(publ + r);
#pragma unroll
            for (int c = 0; c < RES_COLS; ++c) {
                const float xr = c == RES_COLS - 1 ? br : xs[q][c + 1];
                float xn, yn;
                update_elem(xs[q][c], ys[q][c], acc[c], hv, prev, xr, jp_n, kA_n, a.kB, a.dt, a.kD, xn, yn);
                const uint32_t f = ternary_byte(xn, d);
                if (c < 4) lo |= f << (8 * c);
                else hi |= f << (8 * (c - 4));
                prev = xs[q][c];
                xs[q][c] = xn;
                ys[q][c] = yn;
            }
            fnew[q] = make_uint2(lo, hi);
            // keep rows apart in the schedule: hoisting every row's gathers
            // ahead raises the register demand past two waves per SIMD
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();  // every wave is done reading the step-n operand
        float *pf = slot((n + 1) & 1, w, 0), *pl = slot((n + 1) & 1, w, 1);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int r = t + q * RES_THREADS;
            asm volatile("" : "+v"(r));
            op[r] = fnew[q];
            publish(pf + r, xs[q][0]);
            publish(pl + r, xs[q][RES_COLS - 1]);
        }
        __builtin_amdgcn_s_waitcnt(0);  // this wave's edge stores have completed
        __syncthreads();
        if (t == 0) {
            __hip_atomic_store(a.flags + w, n + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            wait_neighbours(a.flags, wl, wr, n + 1, a.err);
        }
        __syncthreads();
    }

    // write back the state and the operand of the own columns (the row index
    // is passed through an empty asm so these addresses are recomputed here
    // rather than kept live across the step loop)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        int r = t + q * RES_THREADS;
        asm volatile("" : "+v"(r));
        float *xrow = a.x + (int64_t)r * a.Cs + c0;
        float *yrow = a.y + (int64_t)r * a.Cs + c0;
        *reinterpret_cast<float4 *>(xrow) = make_float4(xs[q][0], xs[q][1], xs[q][2], xs[q][3]);
        *reinterpret_cast<float4 *>(xrow + 4) = make_float4(xs[q][4], xs[q][5], xs[q][6], xs[q][7]);
        *reinterpret_cast<float4 *>(yrow) = make_float4(ys[q][0], ys[q][1], ys[q][2], ys[q][3]);
        *reinterpret_cast<float4 *>(yrow + 4) = make_float4(ys[q][4], ys[q][5], ys[q][6], ys[q][7]);
        *reinterpret_cast<uint2 *>(a.g + (int64_t)r * a.Cs + c0) = op[r];
    }
}

}  // namespace

int resident_degree(int maxdeg) {
    const int opts[] = {4, 6, 8, 12, 16};
    for (int d : opts)
        if (maxdeg <= d) return d;
    return -1;
}

// rows of the resident kernel (N padded to RPT*RES_THREADS)
int resident_rows(int N) {
    const int rpt = resident_rpt(N);
    return rpt < 0 ? -1 : rpt * RES_THREADS;
}

size_t resident_lds_bytes(int N, int D) {
    const int rows = resident_rows(N);
    return rows < 0 ? 0 : (size_t)rows * (8 + 4 * (D + 1));
}

// rows per thread (1, 2, 4 or 8), or -1 when N is too large
int resident_rpt(int N) {
    const int need = (N + RES_THREADS - 1) / RES_THREADS;
    for (int r = 1; r <= RES_MAX_RPT; r *= 2)
        if (need <= r) return r;
    return -1;
}

int resident_cols() { return RES_COLS; }
int resident_threads() { return RES_THREADS; }

template <int RPT, int D>
static hipError_t launch_res(const ResidentArgs &a, int nwg, hipStream_t st) {
    const void *fn = reinterpret_cast<const void *>(&k_csr_resident<RPT, D>);
    const size_t lds = resident_lds_bytes(a.N, D);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    ResidentArgs arg = a;
    void *args[] = {&arg};
    return hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(RES_THREADS), args, (unsigned)lds, st);
}

template <int RPT>
static hipError_t launch_res_d(const ResidentArgs &a, int D, int nwg, hipStream_t st) {
    switch (D) {
        case 4: return launch_res<RPT, 4>(a, nwg, st);
        case 6: return launch_res<RPT, 6>(a, nwg, st);
        case 8: return launch_res<RPT, 8>(a, nwg, st);
        case 12: return launch_res<RPT, 12>(a, nwg, st);
        case 16: return launch_res<RPT, 16>(a, nwg, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_csr_resident(const ResidentArgs &a, int D, hipStream_t st) {
    const int rpt = resident_rpt(a.N);
    if (a.R % RES_COLS || a.Cs % RES_COLS || rpt < 0 || a.N > 65535) return hipErrorInvalidValue;
    const int nwg = a.nwg;
    switch (rpt) {
        case 1: return launch_res_d<1>(a, D, nwg, st);
        case 2: return launch_res_d<2>(a, D, nwg, st);
        case 4: return launch_res_d<4>(a, D, nwg, st);
        case 8: return launch_res_d<8>(a, D, nwg, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t resident_max_blocks(int D, int N, int *blocks_per_cu) {
    const int rpt = resident_rpt(N);
    const size_t lds = resident_lds_bytes(N, D);
    hipError_t e;
#define SBQA_OCC(R_, D_)                                                                                   \
    do {                                                                                                    \
        const void *f_ = reinterpret_cast<const void *>(&k_csr_resident<R_, D_>);                          \
        e = hipFuncSetAttribute(f_, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                  \
        if (e == hipSuccess)                                                                                \
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f_, RES_THREADS, lds);          \
    } while (0)
#define SBQA_OCC_D(R_)                                                                                     \
    switch (D) {                                                                                            \
        case 4: SBQA_OCC(R_, 4); break;                                                                     \
        case 6: SBQA_OCC(R_, 6); break;                                                                     \
        case 8: SBQA_OCC(R_, 8); break;                                                                     \
        case 12: SBQA_OCC(R_, 12); break;                                                                   \
        case 16: SBQA_OCC(R_, 16); break;                                                                   \
        default: e = hipErrorInvalidValue;                                                                  \
    }
    switch (rpt) {
        case 1: SBQA_OCC_D(1) break;
        case 2: SBQA_OCC_D(2) break;
        case 4: SBQA_OCC_D(4) break;
        case 8: SBQA_OCC_D(8) break;
        default: e = hipErrorInvalidValue;
    }
#undef SBQA_OCC_D
#undef SBQA_OCC
    return e;
}

}  // namespace sbqa
