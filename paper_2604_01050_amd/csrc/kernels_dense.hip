// Dense SBQA kernels for gfx950 (CDNA4, wave64):
//   * the coupling sum of Eq. 7 as an MFMA GEMM over all runs and replicas,
//     Phi^T[c][i] = sum_j f(X)^T[c][j] J[i][j]  (J symmetric, zero diagonal),
//     in fp32, e4m3 fp8, bf16 hi+lo (three products) or fp64 (energies);
//   * the fused update of Eqs. 6-7 (pump, Trotter ring, kick, drift, wall)
//     that also emits the next contraction operand f(X) (Eq. 8).
// State and operands are replica-major ([C][Np]): both GEMM operands are then
// K-contiguous and the update streams rows of Np spins.
#include "sbqa_internal.h"

namespace sbqa {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int LDS_STRIDE = GEMM_KB + 16;  // padded LDS row (bytes): spreads rows over banks
constexpr int TILE_BYTES = GEMM_BM * LDS_STRIDE;
static_assert(GEMM_BM == GEMM_BN, "square block tile assumed by the loaders");

// e4m3 encodings of the ternary values.
constexpr uint8_t FP8_P1 = 0x38, FP8_M1 = 0xB8;
// E8M0 block scale 2^(127-127) = 1 for the scaled fp8 MFMA.
constexpr int E8M0_ONE = 127;

struct Frag32 { uint4 lo, hi; };  // 32 contiguous bytes of one LDS row

__device__ __forceinline__ Frag32 lds_frag(const uint8_t *tile, int row, int g) {
    const uint8_t *p = tile + row * LDS_STRIDE + g * 32;
    Frag32 f;
    f.lo = *reinterpret_cast<const uint4 *>(p);
    f.hi = *reinterpret_cast<const uint4 *>(p + 16);
    return f;
}

template <int KIND> struct AccT { typedef f4 T; };
template <> struct AccT<GK_F64> { typedef d4 T; };

// One 16x16 block update with the 32-byte K slices a, b of this lane.
// Lane group g = lane/16 holds the same K slice for A and B, so the products
// pair correctly whatever K order the instruction uses inside a slice.
template <int KIND>
__device__ __forceinline__ void mma(typename AccT<KIND>::T &acc, const Frag32 &a, const Frag32 &b,
                                    const Frag32 &a2, const Frag32 &b2) {
    if constexpr (KIND == GK_F32) {
        const float *af = reinterpret_cast<const float *>(&a);
        const float *bf = reinterpret_cast<const float *>(&b);
#pragma unroll
        for (int t = 0; t < 8; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[t], bf[t], acc, 0, 0, 0);
    } else if constexpr (KIND == GK_F64) {
        const double *ad = reinterpret_cast<const double *>(&a);
        const double *bd = reinterpret_cast<const double *>(&b);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[t], bd[t], acc, 0, 0, 0);
    } else if constexpr (KIND == GK_FP8) {
        i8v av, bv;
        __builtin_memcpy(&av, &a, 32);
        __builtin_memcpy(&bv, &b, 32);
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc, 0, 0, 0, E8M0_ONE, 0,
                                                                E8M0_ONE);
    } else {  // GK_BF16X3: hi*hi + hi*lo + lo*hi
        bf8v ah0, ah1, bh0, bh1, al0, al1, bl0, bl1;
        __builtin_memcpy(&ah0, &a.lo, 16);
        __builtin_memcpy(&ah1, &a.hi, 16);
        __builtin_memcpy(&bh0, &b.lo, 16);
        __builtin_memcpy(&bh1, &b.hi, 16);
        __builtin_memcpy(&al0, &a2.lo, 16);
        __builtin_memcpy(&al1, &a2.hi, 16);
        __builtin_memcpy(&bl0, &b2.lo, 16);
        __builtin_memcpy(&bl1, &b2.hi, 16);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al0, bh0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al1, bh1, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bl0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bl1, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bh0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bh1, acc, 0, 0, 0);
    }
}

// Block tile: GEMM_BM operand rows (m = replica column c) x GEMM_BN J rows
// (n = spin i); 4 waves in 2x2, each wave 64x64 = 4x4 MFMA 16x16 blocks.
// K tiles of GEMM_KB bytes are staged through LDS; the next tile is fetched
// into registers while the current one is multiplied.
template <int KIND>
__global__ __launch_bounds__(GEMM_THREADS) void k_gemm(const uint8_t *__restrict__ A,
                                                       const uint8_t *__restrict__ A2,
                                                       const uint8_t *__restrict__ B,
                                                       const uint8_t *__restrict__ B2,
                                                       void *__restrict__ out, int Np, int Cp,
                                                       int ebytes, int kchunk_bytes) {
    constexpr int NT = (KIND == GK_BF16X3) ? 4 : 2;
    __shared__ __align__(16) uint8_t lds[NT * TILE_BYTES];
    typedef typename AccT<KIND>::T Acc;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int n0 = blockIdx.x * GEMM_BN, m0 = blockIdx.y * GEMM_BM, z = blockIdx.z;
    const int64_t rowbytes = (int64_t)Np * ebytes;
    const int64_t kb0 = (int64_t)z * kchunk_bytes;
    const int ntiles = kchunk_bytes / GEMM_KB;

    uint4 ra[4], rb[4], ra2[4], rb2[4];
    auto gload = [&](int kt) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int q = tid + GEMM_THREADS * p, row = q >> 3, c16 = q & 7;
            const int64_t off = kb0 + (int64_t)kt * GEMM_KB + c16 * 16;
            ra[p] = *reinterpret_cast<const uint4 *>(A + (int64_t)(m0 + row) * rowbytes + off);
            rb[p] = *reinterpret_cast<const uint4 *>(B + (int64_t)(n0 + row) * rowbytes + off);
            if constexpr (KIND == GK_BF16X3) {
                ra2[p] = *reinterpret_cast<const uint4 *>(A2 + (int64_t)(m0 + row) * rowbytes + off);
                rb2[p] = *reinterpret_cast<const uint4 *>(B2 + (int64_t)(n0 + row) * rowbytes + off);
            }
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int q = tid + GEMM_THREADS * p, row = q >> 3, c16 = q & 7;
            const int o = row * LDS_STRIDE + c16 * 16;
            *reinterpret_cast<uint4 *>(lds + o) = ra[p];
            *reinterpret_cast<uint4 *>(lds + TILE_BYTES + o) = rb[p];
            if constexpr (KIND == GK_BF16X3) {
                *reinterpret_cast<uint4 *>(lds + 2 * TILE_BYTES + o) = ra2[p];
                *reinterpret_cast<uint4 *>(lds + 3 * TILE_BYTES + o) = rb2[p];
            }
        }
    };

    Acc acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    const int g = lane >> 4, r16 = lane & 15;
    gload(0);
    for (int kt = 0; kt < ntiles; ++kt) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (kt + 1 < ntiles) gload(kt + 1);
        Frag32 bf[4], bf2[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            bf[nb] = lds_frag(lds + TILE_BYTES, wn * 64 + nb * 16 + r16, g);
            if constexpr (KIND == GK_BF16X3) bf2[nb] = lds_frag(lds + 3 * TILE_BYTES, wn * 64 + nb * 16 + r16, g);
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            Frag32 af = lds_frag(lds, wm * 64 + mb * 16 + r16, g);
            Frag32 af2 = af;
            if constexpr (KIND == GK_BF16X3) af2 = lds_frag(lds + 2 * TILE_BYTES, wm * 64 + mb * 16 + r16, g);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) mma<KIND>(acc[mb][nb], af, bf[nb], af2, bf2[nb]);
        }
    }

    // D[m][n], column lane%16 of each 16x16 block; f32 results: register r is
    // row 4*(lane/16) + r; f64 results: register r is row 4*r + lane/16.
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int mr = (KIND == GK_F64) ? 4 * r + g : 4 * g + r;
                const int m = m0 + wm * 64 + mb * 16 + mr;
                const int n = n0 + wn * 64 + nb * 16 + r16;
                const int64_t o = ((int64_t)z * Cp + m) * Np + n;
                if constexpr (KIND == GK_F64) reinterpret_cast<double *>(out)[o] = acc[mb][nb][r];
                else reinterpret_cast<float *>(out)[o] = acc[mb][nb][r];
            }
}

// ---------------------------------------------------------------------------
// Fused update (Eqs. 6-7 + wall) and operand emission (Eq. 8).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float f_value(int fmode, float x, float delta) {
    if (fmode == 2) return x;                       // bSB
    const float d = (fmode == 1) ? 0.0f : delta;    // dSB: sign(0) = 0
    if (fabsf(x) <= d) return 0.0f;
    return x > 0.0f ? 1.0f : -1.0f;
}

__device__ __forceinline__ uint16_t bf16_rne(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <int PATH>
__device__ __forceinline__ void store_operand(void *g, void *g_lo, int64_t o, float4 f, int fmode) {
    if constexpr (PATH == PATH_F32) {
        *reinterpret_cast<float4 *>(reinterpret_cast<float *>(g) + o) = f;
    } else if constexpr (PATH == PATH_FP8) {
        const float v[4] = {f.x, f.y, f.z, f.w};
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t b = v[e] > 0.0f ? FP8_P1 : (v[e] < 0.0f ? FP8_M1 : 0u);
            w |= b << (8 * e);
        }
        *reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(g) + o) = w;
    } else {  // BF16X3
        const float v[4] = {f.x, f.y, f.z, f.w};
        uint16_t hi[4], lo[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            hi[e] = bf16_rne(v[e]);
            lo[e] = (fmode == 2) ? bf16_rne(v[e] - bf16_to_f32(hi[e])) : (uint16_t)0;
        }
        uint2 H, L;
        H.x = hi[0] | ((uint32_t)hi[1] << 16);
        H.y = hi[2] | ((uint32_t)hi[3] << 16);
        L.x = lo[0] | ((uint32_t)lo[1] << 16);
        L.y = lo[2] | ((uint32_t)lo[3] << 16);
        *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(g) + o) = H;
        *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(g_lo) + o) = L;
    }
}

#pragma clang fp contract(off)
// One thread: 4 consecutive spins i of one replica column c (grid.y = c).
// The ring neighbours are columns r*R + (k -+ 1 mod R) of the same run.
template <int PATH>
__global__ __launch_bounds__(256) void k_dense_update(int N, int Np, int R, int Cp, int splits,
                                                      const float *__restrict__ phi,
                                                      const float *__restrict__ h,
                                                      const float *__restrict__ x_in,
                                                      float *__restrict__ x_out, float *__restrict__ y,
                                                      void *g, void *g_lo, const float *__restrict__ jp,
                                                      int64_t jp_stride, StepCoef k, int fmode) {
    const int c = blockIdx.y;
    const int i4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i4 >= Np) return;
    const int r = c / R, kk = c - r * R;
    const int cl = r * R + (kk == 0 ? R - 1 : kk - 1);
    const int cr = r * R + (kk == R - 1 ? 0 : kk + 1);
    const int64_t o = (int64_t)c * Np + i4;
    const float4 x = *reinterpret_cast<const float4 *>(x_in + o);
    const float4 xl = *reinterpret_cast<const float4 *>(x_in + (int64_t)cl * Np + i4);
    const float4 xr = *reinterpret_cast<const float4 *>(x_in + (int64_t)cr * Np + i4);
    const float4 yv = *reinterpret_cast<const float4 *>(y + o);
    const float4 hv = *reinterpret_cast<const float4 *>(h + i4);
    float4 ph = *reinterpret_cast<const float4 *>(phi + o);
    for (int zz = 1; zz < splits; ++zz) {
        const float4 q = *reinterpret_cast<const float4 *>(phi + ((int64_t)zz * Cp + c) * Np + i4);
        ph.x += q.x; ph.y += q.y; ph.z += q.z; ph.w += q.w;
    }
    const float jpr = jp[(int64_t)r * jp_stride];
    const float xs[4] = {x.x, x.y, x.z, x.w}, ls[4] = {xl.x, xl.y, xl.z, xl.w};
    const float rs[4] = {xr.x, xr.y, xr.z, xr.w}, ys[4] = {yv.x, yv.y, yv.z, yv.w};
    const float hs[4] = {hv.x, hv.y, hv.z, hv.w}, ps[4] = {ph.x, ph.y, ph.z, ph.w};
    float xo[4], yo[4], fo[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float force = (-k.kA * xs[e] + k.kB * (ps[e] + hs[e])) + jpr * (ls[e] + rs[e]);
        float yn = ys[e] + k.dt * force;
        float xn = xs[e] + k.kD * yn;
        if (fabsf(xn) > 1.0f) {
            xn = xn > 0.0f ? 1.0f : -1.0f;
            yn = 0.0f;
        }
        if (i4 + e >= N) { xn = 0.0f; yn = 0.0f; }  // padding stays zero
        xo[e] = xn;
        yo[e] = yn;
        fo[e] = f_value(fmode, xn, k.delta_next);
    }
    *reinterpret_cast<float4 *>(x_out + o) = make_float4(xo[0], xo[1], xo[2], xo[3]);
    *reinterpret_cast<float4 *>(y + o) = make_float4(yo[0], yo[1], yo[2], yo[3]);
    store_operand<PATH>(g, g_lo, o, make_float4(fo[0], fo[1], fo[2], fo[3]), fmode);
}
#pragma clang fp contract(on)

template <int PATH>
__global__ __launch_bounds__(256) void k_dense_operand(int N, int Np, const float *__restrict__ x, void *g,
                                                       void *g_lo, float delta, int fmode) {
    const int c = blockIdx.y;
    const int i4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i4 >= Np) return;
    const int64_t o = (int64_t)c * Np + i4;
    const float4 v = *reinterpret_cast<const float4 *>(x + o);
    float4 f = make_float4(f_value(fmode, v.x, delta), f_value(fmode, v.y, delta),
                           f_value(fmode, v.z, delta), f_value(fmode, v.w, delta));
    (void)N;
    store_operand<PATH>(g, g_lo, o, f, fmode);
}

__global__ __launch_bounds__(256) void k_sum_partials(int Np, int Cp, int splits, const float *__restrict__ phi,
                                                      float *__restrict__ out) {
    const int c = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Np) return;
    float s = phi[(int64_t)c * Np + i];
    for (int zz = 1; zz < splits; ++zz) s += phi[((int64_t)zz * Cp + c) * Np + i];
    out[(int64_t)c * Np + i] = s;
}

}  // namespace

hipError_t launch_gemm(GemmKind kind, const void *A, const void *A2, const void *B, const void *B2,
                       void *out, int Np, int Cp, int splits, hipStream_t st) {
    const int eb = (kind == GK_F32) ? 4 : (kind == GK_FP8) ? 1 : (kind == GK_F64) ? 8 : 2;
    const int64_t kbytes = (int64_t)Np * eb;
    if (Np % GEMM_BN || Cp % GEMM_BM || splits < 1 || kbytes % ((int64_t)splits * GEMM_KB))
        return hipErrorInvalidValue;
    const int kchunk = (int)(kbytes / splits);
    dim3 grid(Np / GEMM_BN, Cp / GEMM_BM, splits), block(GEMM_THREADS);
    const uint8_t *a = static_cast<const uint8_t *>(A), *a2 = static_cast<const uint8_t *>(A2);
    const uint8_t *b = static_cast<const uint8_t *>(B), *b2 = static_cast<const uint8_t *>(B2);
    switch (kind) {
        case GK_F32: hipLaunchKernelGGL(k_gemm<GK_F32>, grid, block, 0, st, a, a2, b, b2, out, Np, Cp, eb, kchunk); break;
        case GK_FP8: hipLaunchKernelGGL(k_gemm<GK_FP8>, grid, block, 0, st, a, a2, b, b2, out, Np, Cp, eb, kchunk); break;
        case GK_BF16X3: hipLaunchKernelGGL(k_gemm<GK_BF16X3>, grid, block, 0, st, a, a2, b, b2, out, Np, Cp, eb, kchunk); break;
        case GK_F64: hipLaunchKernelGGL(k_gemm<GK_F64>, grid, block, 0, st, a, a2, b, b2, out, Np, Cp, eb, kchunk); break;
    }
    return hipGetLastError();
}

hipError_t launch_dense_update(Path path, int fmode, int N, int Np, int R, int runs, int Cp,
                               int splits, const float *phi, const float *h, const float *x_in,
                               float *x_out, float *y, void *g, void *g_lo, const float *jp,
                               int64_t jp_stride, StepCoef k, hipStream_t st) {
    const int C = R * runs;
    dim3 grid((Np / 4 + 255) / 256, C), block(256);
    switch (path) {
        case PATH_F32: hipLaunchKernelGGL(k_dense_update<PATH_F32>, grid, block, 0, st, N, Np, R, Cp, splits, phi, h, x_in, x_out, y, g, g_lo, jp, jp_stride, k, fmode); break;
        case PATH_FP8: hipLaunchKernelGGL(k_dense_update<PATH_FP8>, grid, block, 0, st, N, Np, R, Cp, splits, phi, h, x_in, x_out, y, g, g_lo, jp, jp_stride, k, fmode); break;
        case PATH_BF16X3: hipLaunchKernelGGL(k_dense_update<PATH_BF16X3>, grid, block, 0, st, N, Np, R, Cp, splits, phi, h, x_in, x_out, y, g, g_lo, jp, jp_stride, k, fmode); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dense_operand(Path path, int fmode, int N, int Np, int C, const float *x, void *g,
                                void *g_lo, float delta, hipStream_t st) {
    dim3 grid((Np / 4 + 255) / 256, C), block(256);
    switch (path) {
        case PATH_F32: hipLaunchKernelGGL(k_dense_operand<PATH_F32>, grid, block, 0, st, N, Np, x, g, g_lo, delta, fmode); break;
        case PATH_FP8: hipLaunchKernelGGL(k_dense_operand<PATH_FP8>, grid, block, 0, st, N, Np, x, g, g_lo, delta, fmode); break;
        case PATH_BF16X3: hipLaunchKernelGGL(k_dense_operand<PATH_BF16X3>, grid, block, 0, st, N, Np, x, g, g_lo, delta, fmode); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sum_partials(int N, int Np, int C, int Cp, int splits, const float *phi, float *out,
                               hipStream_t st) {
    (void)N;
    dim3 grid((Np + 255) / 256, C), block(256);
    hipLaunchKernelGGL(k_sum_partials, grid, block, 0, st, Np, Cp, splits, phi, out);
    return hipGetLastError();
}

}  // namespace sbqa
