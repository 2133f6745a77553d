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

// Coupling sum of the 4 columns c..c+3 of row i, accumulated in CSR order in
// fp32. The row's neighbours are taken GATHER_BATCH at a time: their indices
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
                    a0 += ws[q] * v[q].x; a1 += ws[q] * v[q].y; a2 += ws[q] * v[q].z; a3 += ws[q] * v[q].w;
                }
        } else {
            uint32_t v[GATHER_BATCH];
#pragma unroll
            for (int q = 0; q < GATHER_BATCH; ++q)
                if (q < cnt) v[q] = *reinterpret_cast<const uint32_t *>(g_in + (int64_t)js[q] * Cs + c);
#pragma unroll
            for (int q = 0; q < GATHER_BATCH; ++q)
                if (q < cnt) {
                    a0 += ws[q] * (float)(int8_t)(v[q] & 0xFF);
                    a1 += ws[q] * (float)(int8_t)((v[q] >> 8) & 0xFF);
                    a2 += ws[q] * (float)(int8_t)((v[q] >> 16) & 0xFF);
                    a3 += ws[q] * (float)(int8_t)(v[q] >> 24);
                }
        }
    }
    return make_float4(a0, a1, a2, a3);
}

#pragma clang fp contract(off)
// RING_SHFL: R divides 256 and is a multiple of 4, so every run lies inside
// one wavefront's 256 columns and its R/4 lanes; the ring neighbours outside a
// lane's 4 columns come from the adjacent lane of the same run by a cross-lane
// read. Otherwise they are read from the row in memory.
template <bool BALLISTIC, bool RING_SHFL>
__global__ __launch_bounds__(256) void k_csr_step(int N, int Cs, int C, int R, int nchunk,
                                                  const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col,
                                                  const float *__restrict__ val, const float *__restrict__ h,
                                                  const float *__restrict__ x_in, float *__restrict__ x_out,
                                                  float *__restrict__ y, const int8_t *__restrict__ g_in,
                                                  int8_t *__restrict__ g_out, const float *__restrict__ jp,
                                                  int64_t jp_stride, StepCoef k, int fmode) {
    const int b = blockIdx.x;
    const int chunk = b % nchunk, rg = b / nchunk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = rg * WAVES + wave;
    const int c = chunk * COLS_PER_WAVE + lane * 4;
    if (i >= N || c >= C) return;

    const int64_t o = (int64_t)i * Cs + c;
    const float4 x = *reinterpret_cast<const float4 *>(x_in + o);
    const float4 yv = *reinterpret_cast<const float4 *>(y + o);
    const float4 phi = gather_fields<BALLISTIC>(i, c, Cs, row_ptr, col, val, x_in, g_in);
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
        const float force = (-k.kA * xs[e] + k.kB * (ps[e] + hi)) + jpr * (xl + xr);
        float yn = ys[e] + k.dt * force;
        float xn = xs[e] + k.kD * yn;
        if (fabsf(xn) > 1.0f) {
            xn = xn > 0.0f ? 1.0f : -1.0f;
            yn = 0.0f;
        }
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
                                                    const float *__restrict__ val, const float *__restrict__ x,
                                                    const int8_t *__restrict__ g, float *__restrict__ phi) {
    const int b = blockIdx.x;
    const int chunk = b % nchunk, rg = b / nchunk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = rg * WAVES + wave;
    const int c = chunk * COLS_PER_WAVE + lane * 4;
    if (i >= N || c >= C) return;
    const float4 v = gather_fields<BALLISTIC>(i, c, Cs, row_ptr, col, val, x, g);
    *reinterpret_cast<float4 *>(phi + (int64_t)i * Cs + c) = v;
}

}  // namespace

hipError_t launch_csr_step(int fmode, int N, int Cs, int R, int runs, const int32_t *row_ptr,
                           const int32_t *col, const float *val, const float *h, const float *x_in,
                           float *x_out, float *y, const int8_t *g_in, int8_t *g_out, const float *jp,
                           int64_t jp_stride, StepCoef k, hipStream_t st) {
    const int C = R * runs;
    if (Cs % 4 || Cs < C) return hipErrorInvalidValue;
    const int nchunk = (C + COLS_PER_WAVE - 1) / COLS_PER_WAVE;
    const int nrg = (N + WAVES - 1) / WAVES;
    dim3 grid(nchunk * nrg), block(WAVES * 64);
    const bool shfl = (R % 4 == 0) && (COLS_PER_WAVE % R == 0);
#define SBQA_CSR_LAUNCH(B, S)                                                                                  \
    hipLaunchKernelGGL((k_csr_step<B, S>), grid, block, 0, st, N, Cs, C, R, nchunk, row_ptr, col, val, h, x_in, \
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

hipError_t launch_csr_operand(int fmode, int N, int Cs, int C, const float *x, int8_t *g, float delta,
                              hipStream_t st) {
    const int64_t n4 = (int64_t)N * Cs / 4;
    dim3 grid((unsigned)((n4 + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_csr_operand, grid, block, 0, st, N, Cs, C, x, g, delta, fmode);
    return hipGetLastError();
}

hipError_t launch_csr_fields(int fmode, int N, int Cs, int C, const int32_t *row_ptr, const int32_t *col,
                             const float *val, const float *x, const int8_t *g, float *phi, hipStream_t st) {
    const int nchunk = (C + COLS_PER_WAVE - 1) / COLS_PER_WAVE;
    const int nrg = (N + WAVES - 1) / WAVES;
    dim3 grid(nchunk * nrg), block(WAVES * 64);
    if (fmode == 2)
        hipLaunchKernelGGL(k_csr_fields<true>, grid, block, 0, st, N, Cs, C, nchunk, row_ptr, col, val, x, g, phi);
    else
        hipLaunchKernelGGL(k_csr_fields<false>, grid, block, 0, st, N, Cs, C, nchunk, row_ptr, col, val, x, g, phi);
    return hipGetLastError();
}

}  // namespace sbqa
