// Sparse (CSR) SBQA step for gfx950: the coupling sum of Eq. 7 over the
// neighbours of spin i, fused with the update of Eqs. 6-7 (pump, Trotter ring,
// kick, drift, wall) and the emission of the next operand f(X) (Eq. 8).
//
// State is spin-major ([N][Cs], Cs = C rounded up to 4): one wavefront owns
// one spin row i and 256 consecutive replica columns (4 per lane), so every
// neighbour gather is one contiguous 256-byte (int8 operand) or 1 KiB (fp32
// ballistic operand) read. Blocks are numbered so that block b handles column
// chunk b % nchunk: with the round-robin block-to-XCD dispatch, the chunks of
// one XCD stay in its L2 and the gathers hit there.
#include "sbqa_internal.h"

namespace sbqa {
namespace {

constexpr int COLS_PER_WAVE = 256;
constexpr int WAVES = 4;

__device__ __forceinline__ float f_value(int fmode, float x, float delta) {
    if (fmode == 2) return x;
    const float d = (fmode == 1) ? 0.0f : delta;
    if (fabsf(x) <= d) return 0.0f;
    return x > 0.0f ? 1.0f : -1.0f;
}

__device__ __forceinline__ uint32_t pack_ternary(float a, float b, float c, float d) {
    auto q = [](float v) -> uint32_t { return (uint32_t)(uint8_t)(int8_t)(v > 0.0f ? 1 : (v < 0.0f ? -1 : 0)); };
    return q(a) | (q(b) << 8) | (q(c) << 16) | (q(d) << 24);
}

// Update of one element (Eqs. 6-7 and the wall): kick with the pump term, the
// coupling sum plus field and the ring, then drift, then clamp. Shared by both
// CSR kernels so that they produce identical bits.
__device__ __forceinline__ void update_elem(float x, float y, float phi, float hv, float xl, float xr, float jpr,
                                            float kA, float kB, float dt, float kD, float &xo, float &yo) {
#pragma clang fp contract(off)
    // force = -kA x + kB (phi + h) + J_perp (x_left + x_right), with explicit
    // fused multiply-adds so every kernel that calls this rounds identically
    const float force = __builtin_fmaf(jpr, xl + xr, __builtin_fmaf(kB, phi + hv, -kA * x));
    float yn = __builtin_fmaf(dt, force, y);
    float xn = __builtin_fmaf(kD, yn, x);
    if (fabsf(xn) > 1.0f) {
        xn = xn > 0.0f ? 1.0f : -1.0f;
        yn = 0.0f;
    }
    xo = xn;
    yo = yn;
}

__device__ __forceinline__ uint32_t ternary_byte(float x, float d) {
    return (uint32_t)(uint8_t)(int8_t)(x > d ? 1 : (x < -d ? -1 : 0));
}

// Coupling sum of the 4 columns c..c+3 of row i, accumulated in CSR order in
// fp32 with explicit fused multiply-adds. The row's neighbours are taken GATHER_BATCH at a time: their indices
// and weights are wave-uniform (scalar loads), and all gathers of a batch are
// issued before the first is consumed so their latencies overlap.
constexpr int GATHER_BATCH = 8;

template <bool BALLISTIC>
__device__ __forceinline__ float4 gather_fields(int i, int c, int Cs, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col, const float *__restrict__ val,
                                                const float *__restrict__ x_in, const int8_t *__restrict__ g_in) {
    const int p0 = __builtin_amdgcn_readfirstlane(row_ptr[i]);
    const int p1 = __builtin_amdgcn_readfirstlane(row_ptr[i + 1]);
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int p = p0; p < p1; p += GATHER_BATCH) {
        const int cnt = min(GATHER_BATCH, p1 - p);
        int js[GATHER_BATCH];
        float ws[GATHER_BATCH];
#pragma unroll
        for (int q = 0; q < GATHER_BATCH; ++q) {
            js[q] = q < cnt ? col[p + q] : 0;
            ws[q] = q < cnt ? val[p + q] : 0.f;
        }
        if constexpr (BALLISTIC) {
            float4 v[GATHER_BATCH];
#pragma unroll
            for (int q = 0; q < GATHER_BATCH; ++q)
                if (q < cnt) v[q] = *reinterpret_cast<const float4 *>(x_in + (int64_t)js[q] * Cs + c);
#pragma unroll
            for (int q = 0; q < GATHER_BATCH; ++q)
                if (q < cnt) {
                    a0 = __builtin_fmaf(ws[q], v[q].x, a0);
                    a1 = __builtin_fmaf(ws[q], v[q].y, a1);
                    a2 = __builtin_fmaf(ws[q], v[q].z, a2);
                    a3 = __builtin_fmaf(ws[q], v[q].w, a3);
                }
        } else {
            uint32_t v[GATHER_BATCH];
#pragma unroll
            for (int q = 0; q < GATHER_BATCH; ++q)
                if (q < cnt) v[q] = *reinterpret_cast<const uint32_t *>(g_in + (int64_t)js[q] * Cs + c);
#pragma unroll
            for (int q = 0; q < GATHER_BATCH; ++q)
                if (q < cnt) {
                    a0 = __builtin_fmaf(ws[q], (float)(int8_t)(v[q] & 0xFF), a0);
                    a1 = __builtin_fmaf(ws[q], (float)(int8_t)((v[q] >> 8) & 0xFF), a1);
                    a2 = __builtin_fmaf(ws[q], (float)(int8_t)((v[q] >> 16) & 0xFF), a2);
                    a3 = __builtin_fmaf(ws[q], (float)(int8_t)(v[q] >> 24), a3);
                }
        }
    }
    return make_float4(a0, a1, a2, a3);
}

// Three-body coupling sums of the 4 columns c..c+3 of row i (the cubic term
// of Eq. 11), continuing the accumulators acc: for each triple containing i,
// in list order, acc += K f_a f_b with the other two members' operands (the
// product f_a f_b is exact for ternary operands).
template <bool BALLISTIC>
__device__ __forceinline__ float4 gather_fields3(int i, int c, int Cs, const Tri3 &t3, const float *__restrict__ x_in,
                                                 const int8_t *__restrict__ g_in, float4 acc) {
    const int p0 = __builtin_amdgcn_readfirstlane(t3.ptr[i]);
    const int p1 = __builtin_amdgcn_readfirstlane(t3.ptr[i + 1]);
    constexpr int B = GATHER_BATCH / 2;
    float a[4] = {acc.x, acc.y, acc.z, acc.w};
    for (int p = p0; p < p1; p += B) {
        const int cnt = min(B, p1 - p);
        int ja[B], jb[B];
        float ws[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
            ja[q] = q < cnt ? t3.ab[2 * (p + q)] : 0;
            jb[q] = q < cnt ? t3.ab[2 * (p + q) + 1] : 0;
            ws[q] = q < cnt ? t3.k[p + q] : 0.f;
        }
        if constexpr (BALLISTIC) {
            float4 va[B], vb[B];
#pragma unroll
            for (int q = 0; q < B; ++q)
                if (q < cnt) {
                    va[q] = *reinterpret_cast<const float4 *>(x_in + (int64_t)ja[q] * Cs + c);
                    vb[q] = *reinterpret_cast<const float4 *>(x_in + (int64_t)jb[q] * Cs + c);
                }
#pragma unroll
            for (int q = 0; q < B; ++q)
                if (q < cnt) {
                    const float pa[4] = {va[q].x, va[q].y, va[q].z, va[q].w};
                    const float pb[4] = {vb[q].x, vb[q].y, vb[q].z, vb[q].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float prod = pa[e] * pb[e];
                        a[e] = __builtin_fmaf(ws[q], prod, a[e]);
                    }
                }
        } else {
            uint32_t va[B], vb[B];
#pragma unroll
            for (int q = 0; q < B; ++q)
                if (q < cnt) {
                    va[q] = *reinterpret_cast<const uint32_t *>(g_in + (int64_t)ja[q] * Cs + c);
                    vb[q] = *reinterpret_cast<const uint32_t *>(g_in + (int64_t)jb[q] * Cs + c);
                }
#pragma unroll
            for (int q = 0; q < B; ++q)
                if (q < cnt) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int prod = (int)(int8_t)(va[q] >> (8 * e)) * (int)(int8_t)(vb[q] >> (8 * e));
                        a[e] = __builtin_fmaf(ws[q], (float)prod, a[e]);
                    }
                }
        }
    }
    return make_float4(a[0], a[1], a[2], a[3]);
}

#pragma clang fp contract(off)
// RING_SHFL: R divides 256 and is a multiple of 4, so every run lies inside
// one wavefront's 256 columns and its R/4 lanes; the ring neighbours outside a
// lane's 4 columns come from the adjacent lane of the same run by a cross-lane
// read. Otherwise they are read from the row in memory.
template <bool BALLISTIC, bool RING_SHFL>
__device__ __forceinline__ void csr_step_body(int b, int N, int Cs, int C, int R, int nchunk,
                                              const int32_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ col,
                                              const float *__restrict__ val, const Tri3 &t3,
                                              const float *__restrict__ h,
                                              const float *__restrict__ x_in, float *__restrict__ x_out,
                                              float *__restrict__ y, const int8_t *__restrict__ g_in,
                                              int8_t *__restrict__ g_out, const float *__restrict__ jp,
                                              int64_t jp_stride, StepCoef k, int fmode) {
    const int chunk = b % nchunk, rg = b / nchunk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = rg * WAVES + wave;
    const int c = chunk * COLS_PER_WAVE + lane * 4;
    if (i >= N || c >= C) return;

    const int64_t o = (int64_t)i * Cs + c;
    const float4 x = *reinterpret_cast<const float4 *>(x_in + o);
    const float4 yv = *reinterpret_cast<const float4 *>(y + o);
    float4 phi = gather_fields<BALLISTIC>(i, c, Cs, row_ptr, col, val, x_in, g_in);
    if (t3.ptr) phi = gather_fields3<BALLISTIC>(i, c, Cs, t3, x_in, g_in, phi);
    const float hi = h[i];
    const float xs[4] = {x.x, x.y, x.z, x.w}, ys[4] = {yv.x, yv.y, yv.z, yv.w};
    const float ps[4] = {phi.x, phi.y, phi.z, phi.w};
    float left0 = 0.f, right3 = 0.f;
    if constexpr (RING_SHFL) {
        const int R4 = R >> 2, kq = (c % R) >> 2;
        const int src_l = kq == 0 ? lane + R4 - 1 : lane - 1;
        const int src_r = kq == R4 - 1 ? lane - R4 + 1 : lane + 1;
        left0 = __shfl(xs[3], src_l);
        right3 = __shfl(xs[0], src_r);
    }
    const float *xrow = x_in + (int64_t)i * Cs;
    float xo[4], yo[4], fo[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int cc = c + e;
        if (!RING_SHFL && cc >= C) { xo[e] = xs[e]; yo[e] = ys[e]; fo[e] = 0.f; continue; }
        const int r = cc / R, kk = cc - r * R;
        float xl, xr;
        if constexpr (RING_SHFL) {
            xl = e == 0 ? left0 : xs[e - 1];
            xr = e == 3 ? right3 : xs[e + 1];
            if (R == 4) { xl = xs[(e + 3) & 3]; xr = xs[(e + 1) & 3]; }
        } else {
            const int cl = r * R + (kk == 0 ? R - 1 : kk - 1);
            const int cr = r * R + (kk == R - 1 ? 0 : kk + 1);
            xl = (cl >= c && cl < c + 4) ? xs[cl - c] : xrow[cl];
            xr = (cr >= c && cr < c + 4) ? xs[cr - c] : xrow[cr];
        }
        const float jpr = jp[(int64_t)r * jp_stride];
        float xn, yn;
        update_elem(xs[e], ys[e], ps[e], hi, xl, xr, jpr, k.kA, k.kB, k.dt, k.kD, xn, yn);
        xo[e] = xn;
        yo[e] = yn;
        fo[e] = f_value(fmode, xn, k.delta_next);
    }
    *reinterpret_cast<float4 *>(x_out + o) = make_float4(xo[0], xo[1], xo[2], xo[3]);
    *reinterpret_cast<float4 *>(y + o) = make_float4(yo[0], yo[1], yo[2], yo[3]);
    if constexpr (!BALLISTIC)
        *reinterpret_cast<uint32_t *>(g_out + o) = pack_ternary(fo[0], fo[1], fo[2], fo[3]);
}
#pragma clang fp contract(on)

template <bool BALLISTIC, bool RING_SHFL>
__global__ __launch_bounds__(256) void k_csr_step(int N, int Cs, int C, int R, int nchunk,
                                                  const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col,
                                                  const float *__restrict__ val, const Tri3 t3,
                                                  const float *__restrict__ h,
                                                  const float *__restrict__ x_in, float *__restrict__ x_out,
                                                  float *__restrict__ y, const int8_t *__restrict__ g_in,
                                                  int8_t *__restrict__ g_out, const float *__restrict__ jp,
                                                  int64_t jp_stride, StepCoef k, int fmode) {
    csr_step_body<BALLISTIC, RING_SHFL>(blockIdx.x, N, Cs, C, R, nchunk, row_ptr, col, val, t3, h, x_in, x_out, y,
                                        g_in, g_out, jp, jp_stride, k, fmode);
}

// Grouped step of every CSR instance of one serving group: a grid-stride loop
// over the virtual blocks of all tasks (task q owns blocks [first, first +
// nblocks)), each running exactly the block of the standalone kernel for the
// task's step n = n_base + offset; tasks past their last step skip.
template <bool BALLISTIC, bool RING_SHFL>
__global__ __launch_bounds__(256) void k_group_csr(const GroupHeader *__restrict__ hdr,
                                                   const GroupTask *__restrict__ tasks, int offset) {
    const int ntask = hdr->ntask, total = hdr->total_blocks;
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        int q = 0;
        while (q + 1 < ntask && tasks[q + 1].first_block <= vb) ++q;
        const GroupTask &t = tasks[q];
        const int n = t.n_base + offset;
        if (n >= t.n_end) continue;
        const int in = n & 1;
        StepCoef k;
        k.kA = t.coefA[n];
        k.kB = t.kB;
        k.dt = t.dt;
        k.kD = t.kD;
        k.delta_next = t.delta[n + 1];
        csr_step_body<BALLISTIC, RING_SHFL>(vb - t.first_block, t.N, t.ld, t.C, t.R, t.nchunk, t.row_ptr, t.col,
                                            t.val, t.t3, t.h, t.x[in], t.x[1 - in], t.y, (const int8_t *)t.g[in],
                                            (int8_t *)t.g[1 - in], t.jp + n, t.S, k, t.fmode);
    }
}

__global__ __launch_bounds__(256) void k_csr_operand(int N, int Cs, int C, const float *__restrict__ x,
                                                     int8_t *__restrict__ g, float delta, int fmode) {
    const int64_t e4 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (e4 >= (int64_t)N * Cs) return;
    const int c = (int)(e4 % Cs);
    const float4 v = *reinterpret_cast<const float4 *>(x + e4);
    float f[4] = {f_value(fmode, v.x, delta), f_value(fmode, v.y, delta), f_value(fmode, v.z, delta),
                  f_value(fmode, v.w, delta)};
    for (int e = 0; e < 4; ++e)
        if (c + e >= C) f[e] = 0.f;
    *reinterpret_cast<uint32_t *>(g + e4) = pack_ternary(f[0], f[1], f[2], f[3]);
}

template <bool BALLISTIC>
__global__ __launch_bounds__(256) void k_csr_fields(int N, int Cs, int C, int nchunk,
                                                    const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const float *__restrict__ val, const Tri3 t3,
                                                    const float *__restrict__ x, const int8_t *__restrict__ g,
                                                    float *__restrict__ phi) {
    const int b = blockIdx.x;
    const int chunk = b % nchunk, rg = b / nchunk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = rg * WAVES + wave;
    const int c = chunk * COLS_PER_WAVE + lane * 4;
    if (i >= N || c >= C) return;
    float4 v = gather_fields<BALLISTIC>(i, c, Cs, row_ptr, col, val, x, g);
    if (t3.ptr) v = gather_fields3<BALLISTIC>(i, c, Cs, t3, x, g, v);
    *reinterpret_cast<float4 *>(phi + (int64_t)i * Cs + c) = v;
}


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

hipError_t launch_csr_step(int fmode, int N, int Cs, int R, int runs, const int32_t *row_ptr,
                           const int32_t *col, const float *val, const Tri3 &t3, const float *h, const float *x_in,
                           float *x_out, float *y, const int8_t *g_in, int8_t *g_out, const float *jp,
                           int64_t jp_stride, StepCoef k, hipStream_t st) {
    const int C = R * runs;
    if (Cs % 4 || Cs < C) return hipErrorInvalidValue;
    const int nchunk = csr_step_chunks(C);
    dim3 grid(csr_step_blocks(N, C)), block(WAVES * 64);
    const bool shfl = csr_ring_shfl(R);
#define SBQA_CSR_LAUNCH(B, S)                                                                                  \
    hipLaunchKernelGGL((k_csr_step<B, S>), grid, block, 0, st, N, Cs, C, R, nchunk, row_ptr, col, val, t3, h, x_in, \
                       x_out, y, g_in, g_out, jp, jp_stride, k, fmode)
    if (fmode == 2) {
        if (shfl) SBQA_CSR_LAUNCH(true, true);
        else SBQA_CSR_LAUNCH(true, false);
    } else {
        if (shfl) SBQA_CSR_LAUNCH(false, true);
        else SBQA_CSR_LAUNCH(false, false);
    }
#undef SBQA_CSR_LAUNCH
    return hipGetLastError();
}

int csr_step_blocks(int N, int C) {
    return ((C + COLS_PER_WAVE - 1) / COLS_PER_WAVE) * ((N + WAVES - 1) / WAVES);
}

int csr_step_chunks(int C) { return (C + COLS_PER_WAVE - 1) / COLS_PER_WAVE; }

bool csr_ring_shfl(int R) { return (R % 4 == 0) && (COLS_PER_WAVE % R == 0); }

hipError_t launch_group_csr(bool ballistic, bool shfl, const GroupHeader *hdr, const GroupTask *tasks, int grid,
                            int offset, hipStream_t st) {
    if (grid < 1) return hipErrorInvalidValue;
#define SBQA_GCSR(B, S) hipLaunchKernelGGL((k_group_csr<B, S>), dim3(grid), dim3(WAVES * 64), 0, st, hdr, tasks, offset)
    if (ballistic) {
        if (shfl) SBQA_GCSR(true, true);
        else SBQA_GCSR(true, false);
    } else {
        if (shfl) SBQA_GCSR(false, true);
        else SBQA_GCSR(false, false);
    }
#undef SBQA_GCSR
    return hipGetLastError();
}

hipError_t launch_csr_operand(int fmode, int N, int Cs, int C, const float *x, int8_t *g, float delta,
                              hipStream_t st) {
    const int64_t n4 = (int64_t)N * Cs / 4;
    dim3 grid((unsigned)((n4 + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_csr_operand, grid, block, 0, st, N, Cs, C, x, g, delta, fmode);
    return hipGetLastError();
}

hipError_t launch_csr_fields(int fmode, int N, int Cs, int C, const int32_t *row_ptr, const int32_t *col,
                             const float *val, const Tri3 &t3, const float *x, const int8_t *g, float *phi,
                             hipStream_t st) {
    const int nchunk = (C + COLS_PER_WAVE - 1) / COLS_PER_WAVE;
    const int nrg = (N + WAVES - 1) / WAVES;
    dim3 grid(nchunk * nrg), block(WAVES * 64);
    if (fmode == 2)
        hipLaunchKernelGGL(k_csr_fields<true>, grid, block, 0, st, N, Cs, C, nchunk, row_ptr, col, val, t3, x, g, phi);
    else
        hipLaunchKernelGGL(k_csr_fields<false>, grid, block, 0, st, N, Cs, C, nchunk, row_ptr, col, val, t3, x, g, phi);
    return hipGetLastError();
}


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
