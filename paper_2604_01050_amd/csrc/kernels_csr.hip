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
#include "csr_common.h"

namespace sbqa {
namespace {

constexpr int COLS_PER_WAVE = 256;
constexpr int WAVES = 4;
using namespace csr;

// Rows per wavefront, as a shift: a wave of 64 lanes x 4 columns covers 256
// replica columns; for C <= 128 it takes 2 rows (C <= 64: 4, C <= 32: 8), one
// per group of 64 >> s lanes, so that every lane carries data.
__device__ __host__ __forceinline__ int csr_rpw_shift(int C) {
    int s = 0;
    while (s < 3 && (COLS_PER_WAVE >> (s + 1)) >= C) ++s;
    return s;
}

// Row and first column of a lane of block b (nchunk column chunks).
struct CsrPos {
    int i, c;
};
__device__ __forceinline__ CsrPos csr_pos(int b, int C, int nchunk) {
    const int s = csr_rpw_shift(C), lpr = 64 >> s;
    const int chunk = b % nchunk, rg = b / nchunk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    return CsrPos{((rg * WAVES + wave) << s) + (lane >> (6 - s)), chunk * COLS_PER_WAVE + 4 * (lane & (lpr - 1))};
}

// Coupling sum of the 4 columns c..c+3 of row i, accumulated in CSR order in
// fp32 with explicit fused multiply-adds. The row's neighbours are taken
// GATHER_BATCH at a time (UNI: the row is wave-uniform, so its indices and
// weights come from scalar loads), and all gathers of a batch are issued
// before the first is consumed so their latencies overlap.
constexpr int GATHER_BATCH = 8;

template <bool BALLISTIC, bool UNI = true>
__device__ __forceinline__ float4 gather_fields(int i, int c, int Cs, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col, const float *__restrict__ val,
                                                const float *__restrict__ x_in, const int8_t *__restrict__ g_in) {
    const int p0 = UNI ? __builtin_amdgcn_readfirstlane(row_ptr[i]) : row_ptr[i];
    const int p1 = UNI ? __builtin_amdgcn_readfirstlane(row_ptr[i + 1]) : row_ptr[i + 1];
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
template <bool BALLISTIC, bool UNI = true>
__device__ __forceinline__ float4 gather_fields3(int i, int c, int Cs, const Tri3 &t3, const float *__restrict__ x_in,
                                                 const int8_t *__restrict__ g_in, float4 acc) {
    const int p0 = UNI ? __builtin_amdgcn_readfirstlane(t3.ptr[i]) : t3.ptr[i];
    const int p1 = UNI ? __builtin_amdgcn_readfirstlane(t3.ptr[i + 1]) : t3.ptr[i + 1];
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

// Non-temporal 16-byte load and store of four consecutive floats.
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 nt_load4(const float *p) {
    const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store4(float *p, const float (&v)[4]) {
    __builtin_nontemporal_store(v4f{v[0], v[1], v[2], v[3]}, reinterpret_cast<v4f *>(p));
}

#pragma clang fp contract(off)
// RING_SHFL: R divides 256 and is a multiple of 4, so every run lies inside
// one wavefront's 256 columns and its R/4 lanes; the ring neighbours outside a
// lane's 4 columns come from the adjacent lane of the same run by a cross-lane
// read. Otherwise they are read from the row in memory. NT: the row's own x
// and y stream through non-temporally, so that the cache keeps the gathered
// operand rows (instances whose state is far larger than the caches; the
// ballistic path gathers x itself and never takes it).
template <bool BALLISTIC, bool RING_SHFL, bool NT = false>
__device__ __forceinline__ void csr_step_body(int b, int N, int Cs, int C, int R, int nchunk,
                                              const int32_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ col,
                                              const float *__restrict__ val, const Tri3 &t3,
                                              const float *__restrict__ h,
                                              const float *__restrict__ x_in, float *__restrict__ x_out,
                                              float *__restrict__ y, const int8_t *__restrict__ g_in,
                                              int8_t *__restrict__ g_out, const float *__restrict__ jp,
                                              int64_t jp_stride, StepCoef k, int fmode) {
    const CsrPos pos = csr_pos(b, C, nchunk);
    const int i = pos.i, c = pos.c, lane = threadIdx.x & 63;
    if (i >= N || c >= C) return;

    const int64_t o = (int64_t)i * Cs + c;
    constexpr bool STREAM = NT && !BALLISTIC;
    const float4 x = STREAM ? nt_load4(x_in + o) : *reinterpret_cast<const float4 *>(x_in + o);
    const float4 yv = STREAM ? nt_load4(y + o) : *reinterpret_cast<const float4 *>(y + o);
    float4 phi;
    if (csr_rpw_shift(C) == 0) {
        phi = gather_fields<BALLISTIC, true>(i, c, Cs, row_ptr, col, val, x_in, g_in);
        if (t3.ptr) phi = gather_fields3<BALLISTIC, true>(i, c, Cs, t3, x_in, g_in, phi);
    } else {
        phi = gather_fields<BALLISTIC, false>(i, c, Cs, row_ptr, col, val, x_in, g_in);
        if (t3.ptr) phi = gather_fields3<BALLISTIC, false>(i, c, Cs, t3, x_in, g_in, phi);
    }
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
    if constexpr (STREAM) {
        nt_store4(x_out + o, xo);
        nt_store4(y + o, yo);
    } else {
        *reinterpret_cast<float4 *>(x_out + o) = make_float4(xo[0], xo[1], xo[2], xo[3]);
        *reinterpret_cast<float4 *>(y + o) = make_float4(yo[0], yo[1], yo[2], yo[3]);
    }
    if constexpr (!BALLISTIC)
        *reinterpret_cast<uint32_t *>(g_out + o) = pack_ternary(fo[0], fo[1], fo[2], fo[3]);
}
#pragma clang fp contract(on)

template <bool BALLISTIC, bool RING_SHFL, bool NT>
__global__ __launch_bounds__(256) void k_csr_step(int N, int Cs, int C, int R, int nchunk,
                                                  const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col,
                                                  const float *__restrict__ val, const Tri3 t3,
                                                  const float *__restrict__ h,
                                                  const float *__restrict__ x_in, float *__restrict__ x_out,
                                                  float *__restrict__ y, const int8_t *__restrict__ g_in,
                                                  int8_t *__restrict__ g_out, const float *__restrict__ jp,
                                                  int64_t jp_stride, StepCoef k, int fmode) {
    csr_step_body<BALLISTIC, RING_SHFL, NT>(blockIdx.x, N, Cs, C, R, nchunk, row_ptr, col, val, t3, h, x_in, x_out,
                                            y, g_in, g_out, jp, jp_stride, k, fmode);
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
    const CsrPos pos = csr_pos(blockIdx.x, C, nchunk);
    const int i = pos.i, c = pos.c;
    if (i >= N || c >= C) return;
    float4 v = gather_fields<BALLISTIC, false>(i, c, Cs, row_ptr, col, val, x, g);
    if (t3.ptr) v = gather_fields3<BALLISTIC, false>(i, c, Cs, t3, x, g, v);
    *reinterpret_cast<float4 *>(phi + (int64_t)i * Cs + c) = v;
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
    // x in, x out and y stream through once per step; when they are larger
    // than the last-level cache (256 MiB on MI355X; 192 MiB leaves room for
    // the operand and the CSR), non-temporal accesses keep them from evicting
    // the gathered operand rows. Smaller states are better served cached.
    const bool nt = 3.0 * 4.0 * (double)N * (double)Cs > 192.0 * 1024 * 1024;
#define SBQA_CSR_LAUNCH(B, S, T)                                                                               \
    hipLaunchKernelGGL((k_csr_step<B, S, T>), grid, block, 0, st, N, Cs, C, R, nchunk, row_ptr, col, val, t3, h,    \
                       x_in, x_out, y, g_in, g_out, jp, jp_stride, k, fmode)
    if (fmode == 2) {
        if (shfl) SBQA_CSR_LAUNCH(true, true, false);
        else SBQA_CSR_LAUNCH(true, false, false);
    } else if (nt) {
        if (shfl) SBQA_CSR_LAUNCH(false, true, true);
        else SBQA_CSR_LAUNCH(false, false, true);
    } else {
        if (shfl) SBQA_CSR_LAUNCH(false, true, false);
        else SBQA_CSR_LAUNCH(false, false, false);
    }
#undef SBQA_CSR_LAUNCH
    return hipGetLastError();
}

int csr_step_blocks(int N, int C) {
    const int rows = WAVES << csr_rpw_shift(C);
    return csr_step_chunks(C) * ((N + rows - 1) / rows);
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
    const int nchunk = csr_step_chunks(C);
    dim3 grid(csr_step_blocks(N, C)), block(WAVES * 64);
    if (fmode == 2)
        hipLaunchKernelGGL(k_csr_fields<true>, grid, block, 0, st, N, Cs, C, nchunk, row_ptr, col, val, t3, x, g, phi);
    else
        hipLaunchKernelGGL(k_csr_fields<false>, grid, block, 0, st, N, Cs, C, nchunk, row_ptr, col, val, t3, x, g, phi);
    return hipGetLastError();
}


}  // namespace sbqa
