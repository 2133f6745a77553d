// Dense SBQA kernels for gfx950 (CDNA4, wave64):
//   * one step of the dense path: the coupling sum of Eq. 7 over all runs and
//     replicas, Phi^T[c][i] = sum_j f(X)^T[c][j] J[i][j] (J symmetric, zero
//     diagonal), on MFMA in fp32, e4m3 fp8 or e2m1 fp4 (J as bytes / nibbles
//     or, for J = +-1, one bit per coupling), int8 (integer J) or bf16 hi+lo
//     (three products),
//     with the update of Eqs. 6-7 (pump, Trotter ring, kick, drift, wall) and
//     the next operand f(X) (Eq. 8) fused into its epilogue;
//   * the fp64 GEMM of the energies (Eq. 2 at the corners).
// State is replica-major ([C][Np]); the contraction operands are
// fragment-tiled (see sbqa_internal.h).
#include "sbqa_internal.h"

#include <type_traits>
#include <utility>

namespace sbqa {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// e4m3 and int8 encodings of the ternary values.
constexpr uint8_t FP8_P1 = 0x38, FP8_M1 = 0xB8;
constexpr uint8_t I8_P1 = 0x01, I8_M1 = 0xFF;
// e2m1 (fp4) nibbles of +1 and -1 (sign bit 3, exponent 01, mantissa 0).
constexpr uint32_t FP4_P1 = 0x2, FP4_M1 = 0xA;
// E8M0 block scale 2^(127-127) = 1 for the scaled fp8 MFMA.
constexpr int E8M0_ONE = 127;

struct Frag32 { uint4 lo, hi; };  // the 32 K bytes of one lane for a 16x16 block

template <int PATH> constexpr bool is_fp8 = PATH == PATH_FP8 || PATH == PATH_FP8PK;
template <int PATH> constexpr bool is_fp4 = PATH == PATH_FP4 || PATH == PATH_FP4PK;

// Bit-packed +-1 J: lane l of a fragment owns the dword at 4*l; its bit
// 8*i + k encodes byte i of dword k (k = 0..7) of the lane's 32 fp8 K bytes,
// set for -1. Dword k is then ((w << (7 - k)) & 0x80808080) | e4m3(+1) x 4.
__device__ __forceinline__ Frag32 unpack_pm1(uint32_t w) {
    auto d = [w](int k) { return ((w << (7 - k)) & 0x80808080u) | 0x38383838u; };
    return Frag32{make_uint4(d(0), d(1), d(2), d(3)), make_uint4(d(4), d(5), d(6), d(7))};
}

// The same for fp4: a lane owns two dwords (one per 16-byte half of its 32
// bytes = 64 nibbles); bit 4*i + k of a half's dword encodes nibble i of dword
// k (k = 0..3) of that half, set for -1, so dword k is
// ((w << (3 - k)) & 0x88888888) | e2m1(+1) x 8.
__device__ __forceinline__ Frag32 unpack_pm1_fp4(uint2 w) {
    auto d = [](uint32_t v, int k) { return ((v << (3 - k)) & 0x88888888u) | 0x22222222u; };
    return Frag32{make_uint4(d(w.x, 0), d(w.x, 1), d(w.x, 2), d(w.x, 3)),
                  make_uint4(d(w.y, 0), d(w.y, 1), d(w.y, 2), d(w.y, 3))};
}

// ---------------------------------------------------------------------------
// fp64 energy GEMM (row-major operands staged through LDS).
// ---------------------------------------------------------------------------
constexpr int LDS_STRIDE = GEMM_KB + 16;  // padded LDS row (bytes): spreads rows over banks
constexpr int TILE_BYTES = GEMM_BM * LDS_STRIDE;
static_assert(GEMM_BM == GEMM_BN, "square block tile assumed by the loaders");

__device__ __forceinline__ Frag32 lds_frag(const uint8_t *tile, int row, int g) {
    const uint8_t *p = tile + row * LDS_STRIDE + g * 32;
    Frag32 f;
    f.lo = *reinterpret_cast<const uint4 *>(p);
    f.hi = *reinterpret_cast<const uint4 *>(p + 16);
    return f;
}

// Block tile: GEMM_BM operand rows (m = replica column c) x GEMM_BN J rows
// (n = spin i); 4 waves in 2x2, each wave 64x64 = 4x4 MFMA 16x16 blocks.
// Lane group g = lane/16 holds the same 32-byte K slice for A and B, so the
// products pair correctly whatever K order the instruction uses in a slice.
__global__ __launch_bounds__(GEMM_THREADS) void k_gemm_f64(const uint8_t *__restrict__ A,
                                                           const uint8_t *__restrict__ B,
                                                           double *__restrict__ out, int Np, int Cp,
                                                           int kchunk_bytes) {
    __shared__ __align__(16) uint8_t lds[2 * TILE_BYTES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int n0 = blockIdx.x * GEMM_BN, m0 = blockIdx.y * GEMM_BM, z = blockIdx.z;
    const int64_t rowbytes = (int64_t)Np * 8;
    const int64_t kb0 = (int64_t)z * kchunk_bytes;
    const int ntiles = kchunk_bytes / GEMM_KB;

    uint4 ra[4], rb[4];
    auto gload = [&](int kt) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int q = tid + GEMM_THREADS * p, row = q >> 3, c16 = q & 7;
            const int64_t off = kb0 + (int64_t)kt * GEMM_KB + c16 * 16;
            ra[p] = *reinterpret_cast<const uint4 *>(A + (int64_t)(m0 + row) * rowbytes + off);
            rb[p] = *reinterpret_cast<const uint4 *>(B + (int64_t)(n0 + row) * rowbytes + off);
        }
    };
    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0, 0, 0, 0};

    const int g = lane >> 4, r16 = lane & 15;
    gload(0);
    for (int kt = 0; kt < ntiles; ++kt) {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int q = tid + GEMM_THREADS * p, row = q >> 3, c16 = q & 7;
            const int o = row * LDS_STRIDE + c16 * 16;
            *reinterpret_cast<uint4 *>(lds + o) = ra[p];
            *reinterpret_cast<uint4 *>(lds + TILE_BYTES + o) = rb[p];
        }
        __syncthreads();
        if (kt + 1 < ntiles) gload(kt + 1);
        Frag32 bf[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) bf[nb] = lds_frag(lds + TILE_BYTES, wn * 64 + nb * 16 + r16, g);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const Frag32 af = lds_frag(lds, wm * 64 + mb * 16 + r16, g);
            const double *ad = reinterpret_cast<const double *>(&af);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const double *bd = reinterpret_cast<const double *>(&bf[nb]);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[t], bd[t], acc[mb][nb], 0, 0, 0);
            }
        }
    }
    // D[m][n]: column lane%16 of each 16x16 block; register r is row 4*r + lane/16.
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 64 + mb * 16 + 4 * r + g;
                const int n = n0 + wn * 64 + nb * 16 + r16;
                out[((int64_t)z * Cp + m) * Np + n] = acc[mb][nb][r];
            }
}

// ---------------------------------------------------------------------------
// Operand formats and the fragment-tiled layout.
// ---------------------------------------------------------------------------

// Byte offset of element (row, k) in a fragment-tiled matrix with nkc K chunks
// and groups of G row blocks.
__device__ __forceinline__ int64_t tf_offset(int row, int k, int nkc, int eb, int G) {
    const int kbyte = k * eb;
    const int kc = kbyte >> 7, kb = kbyte & 127, rb = row >> 4;
    const int l = ((kb >> 5) << 4) | (row & 15);
    return (((int64_t)(rb / G) * nkc + kc) * G + rb % G) * FRAG_BYTES + ((kb >> 4) & 1) * 1024 + l * 16 + (kb & 15);
}

// Byte offset of element (row, k) of an operand or J in the path's format
// (fp4: of the byte that holds elements k and k + 1, k even).
template <int PATH>
__device__ __forceinline__ int64_t op_offset(int row, int k, int nkc, int G) {
    if constexpr (is_fp4<PATH>) return tf_offset(row, k >> 1, nkc, 1, G);
    else return tf_offset(row, k, nkc, path_ebytes(Path(PATH)), G);
}

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

// Four consecutive operand values (same row, K positions k..k+3) at byte
// offset o of the fragment-tiled operand (o from tf_offset: the four values
// are contiguous there).
template <int PATH>
__device__ __forceinline__ void store_operand(void *g, void *g_lo, int64_t o, float4 f, int fmode) {
    uint8_t *gb = reinterpret_cast<uint8_t *>(g);
    if constexpr (PATH == PATH_F32) {
        *reinterpret_cast<float4 *>(gb + o) = f;
    } else if constexpr (is_fp8<PATH> || PATH == PATH_I8) {
        constexpr uint32_t P1 = is_fp8<PATH> ? FP8_P1 : I8_P1, M1 = is_fp8<PATH> ? FP8_M1 : I8_M1;
        const float v[4] = {f.x, f.y, f.z, f.w};
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t b = v[e] > 0.0f ? P1 : (v[e] < 0.0f ? M1 : 0u);
            w |= b << (8 * e);
        }
        *reinterpret_cast<uint32_t *>(gb + o) = w;
    } else if constexpr (is_fp4<PATH>) {
        const float v[4] = {f.x, f.y, f.z, f.w};
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= (v[e] > 0.0f ? FP4_P1 : (v[e] < 0.0f ? FP4_M1 : 0u)) << (4 * e);
        *reinterpret_cast<uint16_t *>(gb + o) = (uint16_t)w;
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
        *reinterpret_cast<uint2 *>(gb + o) = H;
        *reinterpret_cast<uint2 *>(reinterpret_cast<uint8_t *>(g_lo) + o) = L;
    }
}

// ---------------------------------------------------------------------------
// MFMA terms of one 16x16 block with the 32 K bytes a (operand) and b (J) of
// this lane (a2, b2: bf16 low parts). Term t of T<PATH>::terms; every block
// accumulates its terms in the same order.
// ---------------------------------------------------------------------------
template <int PATH> struct Terms;
template <> struct Terms<PATH_F32> { static constexpr int n = 8; };     // 8 x 16x16x4 f32
template <> struct Terms<PATH_FP8> { static constexpr int n = 1; };     // 1 x 16x16x128 f8f6f4
template <> struct Terms<PATH_FP8PK> { static constexpr int n = 1; };
template <> struct Terms<PATH_BF16X3> { static constexpr int n = 6; };  // lo*hi, hi*lo, hi*hi x 2 halves
template <> struct Terms<PATH_I8> { static constexpr int n = 2; };      // 2 x 16x16x64 i8 (K halves)
template <> struct Terms<PATH_FP4> { static constexpr int n = 2; };     // 2 x 16x16x128 fp4 (K halves)
template <> struct Terms<PATH_FP4PK> { static constexpr int n = 2; };

template <int PATH, int T>
__device__ __forceinline__ void mma_term(f4 &acc, const Frag32 &a, const Frag32 &b, const Frag32 &a2,
                                         const Frag32 &b2) {
    if constexpr (PATH == PATH_F32) {
        const float *af = reinterpret_cast<const float *>(&a);
        const float *bf = reinterpret_cast<const float *>(&b);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[T], bf[T], acc, 0, 0, 0);
    } else if constexpr (is_fp8<PATH>) {
        i8v av, bv;
        __builtin_memcpy(&av, &a, 32);
        __builtin_memcpy(&bv, &b, 32);
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc, 0, 0, 0, E8M0_ONE, 0, E8M0_ONE);
    } else if constexpr (PATH == PATH_I8) {
        // int32 accumulation, carried in the float accumulator's bits; term T
        // takes the lane's K bytes of half T (each 16x16x64 product pairs the
        // same lane bytes of both operands, so the two halves cover the
        // chunk's 128 K exactly once)
        const uint4 &xs = T ? a.hi : a.lo;
        const uint4 &ys = T ? b.hi : b.lo;
        i4v xv, yv;
        __builtin_memcpy(&xv, &xs, 16);
        __builtin_memcpy(&yv, &ys, 16);
        acc = __builtin_bit_cast(f4, __builtin_amdgcn_mfma_i32_16x16x64_i8(xv, yv, __builtin_bit_cast(i4v, acc), 0, 0, 0));
    } else if constexpr (is_fp4<PATH>) {
        // e2m1 operands (format 4 for A and B): term T takes the lane's 16
        // bytes of half T (64 lanes x 32 nibbles = one 16x128 K block each)
        const uint4 &xs = T ? a.hi : a.lo;
        const uint4 &ys = T ? b.hi : b.lo;
        const i8v xv = {(int)xs.x, (int)xs.y, (int)xs.z, (int)xs.w, 0, 0, 0, 0};
        const i8v yv = {(int)ys.x, (int)ys.y, (int)ys.z, (int)ys.w, 0, 0, 0, 0};
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(xv, yv, acc, 4, 4, 0, E8M0_ONE, 0, E8M0_ONE);
    } else {
        // small products first: lo*hi, hi*lo, then hi*hi; each over both halves
        const Frag32 &x = (T < 2) ? a2 : a;
        const Frag32 &y = (T >= 2 && T < 4) ? b2 : b;
        const uint4 &xs = (T & 1) ? x.hi : x.lo;
        const uint4 &ys = (T & 1) ? y.hi : y.lo;
        bf8v xv, yv;
        __builtin_memcpy(&xv, &xs, 16);
        __builtin_memcpy(&yv, &ys, 16);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xv, yv, acc, 0, 0, 0);
    }
}

template <int PATH> struct Pipe {
    static constexpr int planes = (PATH == PATH_BF16X3) ? 2 : 1;  // bf16: hi and lo
    static constexpr int depth = dense_depth(Path(PATH));          // K chunks in flight
};

__device__ __forceinline__ uint4 ld16(const uint8_t *p) { return *reinterpret_cast<const uint4 *>(p); }

// Field value of one accumulator element (int8 path: the exact int32 sum,
// rounded once to float32).
template <int PATH>
__device__ __forceinline__ float acc_field(float v) {
    if constexpr (PATH == PATH_I8) return (float)__builtin_bit_cast(int, v);
    else return v;
}

// f(integral_constant<int, I>) for I = B..E-1, unrolled at compile time.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------------------
// Fused update (Eqs. 6-7 + wall) and operand emission (Eq. 8) for four
// consecutive spins i4..i4+3 of replica column c, with their fields ph. The
// inputs are gathered first (UpdIn) so that a lane can have the loads of all
// its items in flight before the first store.
// The ring neighbours are columns r*R + (k -+ 1 mod R) of the same run.
// ---------------------------------------------------------------------------
struct UpdIn {
    float4 x, xl, xr, y, h;
    float jp;
};

__device__ __forceinline__ UpdIn update_load(const DenseStepArgs &a, int c, int i4) {
    const int Np = a.Np, R = a.R;
    const int r = c / R, kk = c - r * R;
    const int cl = r * R + (kk == 0 ? R - 1 : kk - 1);
    const int cr = r * R + (kk == R - 1 ? 0 : kk + 1);
    UpdIn u;
    u.x = *reinterpret_cast<const float4 *>(a.x_in + (int64_t)c * Np + i4);
    u.xl = *reinterpret_cast<const float4 *>(a.x_in + (int64_t)cl * Np + i4);
    u.xr = *reinterpret_cast<const float4 *>(a.x_in + (int64_t)cr * Np + i4);
    u.y = *reinterpret_cast<const float4 *>(a.y + (int64_t)c * Np + i4);
    u.h = *reinterpret_cast<const float4 *>(a.h + i4);
    u.jp = a.jp[(int64_t)r * a.jp_stride];
    return u;
}

#pragma clang fp contract(off)
template <int PATH, int MBW>
__device__ __forceinline__ void update_store(const DenseStepArgs &a, int c, int i4, const UpdIn &u, float4 ph) {
    const StepCoef k = a.k;
    const float xs[4] = {u.x.x, u.x.y, u.x.z, u.x.w}, ls[4] = {u.xl.x, u.xl.y, u.xl.z, u.xl.w};
    const float rs[4] = {u.xr.x, u.xr.y, u.xr.z, u.xr.w}, ys[4] = {u.y.x, u.y.y, u.y.z, u.y.w};
    const float hs[4] = {u.h.x, u.h.y, u.h.z, u.h.w}, ps[4] = {ph.x, ph.y, ph.z, ph.w};
    float xo[4], yo[4], fo[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float force = (-k.kA * xs[e] + k.kB * (ps[e] + hs[e])) + u.jp * (ls[e] + rs[e]);
        float yn = ys[e] + k.dt * force;
        float xn = xs[e] + k.kD * yn;
        if (fabsf(xn) > 1.0f) {
            xn = xn > 0.0f ? 1.0f : -1.0f;
            yn = 0.0f;
        }
        if (i4 + e >= a.N) { xn = 0.0f; yn = 0.0f; }  // padding stays zero
        xo[e] = xn;
        yo[e] = yn;
        fo[e] = f_value(a.fmode, xn, k.delta_next);
    }
    const int64_t o = (int64_t)c * a.Np + i4;
    *reinterpret_cast<float4 *>(a.x_out + o) = make_float4(xo[0], xo[1], xo[2], xo[3]);
    *reinterpret_cast<float4 *>(a.y + o) = make_float4(yo[0], yo[1], yo[2], yo[3]);
    store_operand<PATH>(a.g_next, a.g_next_lo, op_offset<PATH>(c, i4, a.nkc, MBW),
                        make_float4(fo[0], fo[1], fo[2], fo[3]), a.fmode);
}
#pragma clang fp contract(on)

// Epilogue of one workgroup tile: transpose each 16 x DENSE_TN block of Phi
// through LDS (lds: at least 4 waves x 16 x (DENSE_TN + 4) floats) so that a
// lane holds 4 consecutive spins of one replica column (f32 MFMA results:
// register r of a lane is row 4*(lane/16) + r, column lane%16); then load
// every input of the lane's items before the first store. wq: the wave's
// index among the 4 waves of the tile's columns (default: its workgroup
// index); the transpose buffer is indexed by the workgroup wave index.
template <int PATH, int MBW, int EPI>
__device__ __forceinline__ void dense_epilogue(const DenseStepArgs &a, f4 (&acc)[MBW][DENSE_TN / 16], int nt, int mchunk,
                                               uint8_t *lds, int wq = -1) {
    constexpr int RBT = DENSE_TN / 16;
    constexpr int TS = DENSE_TN + 4;
    constexpr bool JPK = path_packed(Path(PATH));
    const int lane = threadIdx.x & 63, wt = threadIdx.x >> 6, w = wq < 0 ? wt : wq;
    const int n0 = nt * DENSE_TN;
    const int mb0 = (mchunk * 4 + w) * MBW;
    const int nkc = a.nkc;
    __syncthreads();
    float *T = reinterpret_cast<float *>(lds) + wt * 16 * TS;
    const int g = lane >> 4, r16 = lane & 15;
    constexpr int QPR = DENSE_TN / 4;         // spin quads per row
    constexpr int ITEMS = 16 * QPR / 64;      // (row, quad) items per lane and m-block
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb) {
#pragma unroll
        for (int p = 0; p < RBT; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) T[(4 * g + r) * TS + 16 * p + r16] = acc_field<PATH>(acc[mb][p][r]);
        __syncthreads();
        float4 ph[ITEMS];
        int cc[ITEMS], ii[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int flat = it * 64 + lane, row = flat / QPR, q = flat % QPR;
            ph[it] = *reinterpret_cast<const float4 *>(T + row * TS + 4 * q);
            cc[it] = 16 * (mb0 + mb) + row;
            ii[it] = n0 + 4 * q;
        }
        if constexpr (JPK) {
            // bit-packed J holds +1 on the diagonal and in the padding: take
            // the diagonal term J'_ii f_i = f_i (the operand byte this step
            // read) back out, and zero the fields of padded spins so that
            // their x and f stay 0
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) {
                if (cc[it] >= a.C) continue;
                const uint8_t *fp = a.g + op_offset<PATH>(cc[it], ii[it], nkc, MBW);
                constexpr int BITS = is_fp4<PATH> ? 4 : 8;
                constexpr uint32_t MASK = (1u << BITS) - 1u, SIGN = 1u << (BITS - 1);
                const uint32_t fb = is_fp4<PATH> ? (uint32_t)*reinterpret_cast<const uint16_t *>(fp)
                                                 : *reinterpret_cast<const uint32_t *>(fp);
                float v[4] = {ph[it].x, ph[it].y, ph[it].z, ph[it].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t b = (fb >> (BITS * e)) & MASK;
                    const float f = b == 0u ? 0.0f : ((b & SIGN) ? -1.0f : 1.0f);
                    v[e] = (ii[it] + e < a.N) ? v[e] - f : 0.0f;
                }
                ph[it] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
        if constexpr (EPI == EPI_UPDATE) {
            UpdIn u[ITEMS];
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
                if (cc[it] < a.C) u[it] = update_load(a, cc[it], ii[it]);
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
                if (cc[it] < a.C) update_store<PATH, MBW>(a, cc[it], ii[it], u[it], ph[it]);
        } else {
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
                if (cc[it] < a.C) *reinterpret_cast<float4 *>(a.phi + (int64_t)cc[it] * a.Np + ii[it]) = ph[it];
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
// One dense step. Workgroup tile: DENSE_TN = 64 spins (4 row blocks of J) x
// 64*MBW replica columns. Wave w owns m-blocks [w*MBW, (w+1)*MBW) of the
// column chunk and all 4 J row blocks: every J fragment is read once per step
// and column chunk, shared by the 4 waves through a double-buffered LDS slot
// (wave w stages row block w), while each wave streams its own operand
// fragments straight into registers, Pipe::depth K chunks ahead. reverse = 1
// walks K backwards: alternating the direction every step starts each step on
// the J chunks the previous one touched last.
// ---------------------------------------------------------------------------
// CG column groups of 4 waves share the tile's J staging (CG = 2: a
// 64-spin x 128*MBW-column workgroup of 8 waves reads every J fragment once
// for twice the columns; with two J planes, group cg stages plane cg).
template <int PATH, int MBW, int EPI, int CG = 1>
__device__ __forceinline__ void dense_step_body(const DenseStepArgs &a, int nt, int mchunk_wg) {
    constexpr int PL = Pipe<PATH>::planes;
    constexpr int PD = Pipe<PATH>::depth;
    constexpr int NT = Terms<PATH>::n;
    constexpr int RBT = DENSE_TN / 16;          // J row blocks per tile
    constexpr int SLOT = PL * RBT * FRAG_BYTES;  // J fragments of one K chunk
    constexpr int TS = DENSE_TN + 4;             // epilogue transpose row stride (floats)
    constexpr int TBYTES = 4 * CG * 16 * TS * 4;
    constexpr int LDS_BYTES = (2 * SLOT > TBYTES) ? 2 * SLOT : TBYTES;
    static_assert(CG == 1 || (CG == 2 && PL == 2), "two column groups split the two J planes");
    __shared__ __align__(16) uint8_t lds[LDS_BYTES];

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, w = wv & 3, cg = wv >> 2;
    const int mchunk = mchunk_wg * CG + cg;       // this wave's 64*MBW-column chunk
    const int n0 = nt * DENSE_TN;
    const int mb0 = (mchunk * 4 + w) * MBW;       // first m-block of this wave
    const int nkc = a.nkc;
    const int l16 = lane * 16;
    constexpr bool JPK = path_packed(Path(PATH));   // J as one bit per coupling
    constexpr int JFRAG = JPK ? pk_frag_bytes(Path(PATH)) : FRAG_BYTES;
    using JWord = std::conditional_t<is_fp4<PATH>, uint2, uint32_t>;   // a lane's packed J of one chunk
    constexpr int JCH = RBT * JFRAG;        // J bytes of one tile and K chunk
    constexpr int XCH = MBW * FRAG_BYTES;   // operand bytes of one wave and K chunk

    // this wave stages J row block w of tile nt (both planes); its operand
    // group is m-blocks mb0..mb0+MBW-1
    const int64_t jgrp = (int64_t)nt * nkc * JCH + w * JFRAG + (JPK ? lane * (int)sizeof(JWord) : l16);
    const int64_t xgrp = (int64_t)(mchunk * 4 + w) * nkc * XCH + l16;
    const uint8_t *jsrc = a.J + jgrp;
    const uint8_t *jsrc_lo = (PL == 2) ? a.J_lo + jgrp : jsrc;
    const uint8_t *xsrc = a.g + xgrp;
    const uint8_t *xsrc_lo = (PL == 2) ? a.g_lo + xgrp : xsrc;

    uint4 jr[JPK ? 1 : PD][PL][2];
    JWord jw[JPK ? PD : 1];
    uint4 xr[PD][MBW][PL][2];
    f4 acc[MBW][RBT];
#pragma unroll
    for (int i = 0; i < MBW; ++i)
#pragma unroll
        for (int j = 0; j < RBT; ++j) acc[i][j] = f4{0, 0, 0, 0};

    const int rev = a.reverse;
    auto chunk_at = [&](int kc) -> int64_t { return rev ? nkc - 1 - kc : kc; };
    auto load_j = [&](int s, int kc) {
        const int64_t o = chunk_at(kc) * JCH;
        if constexpr (JPK) {
            jw[s] = *reinterpret_cast<const JWord *>(jsrc + o);
        } else if constexpr (CG == 2) {
            const uint8_t *src = cg ? jsrc_lo : jsrc;
            jr[s][0][0] = ld16(src + o);
            jr[s][0][1] = ld16(src + o + 1024);
        } else {
            jr[s][0][0] = ld16(jsrc + o);
            jr[s][0][1] = ld16(jsrc + o + 1024);
            if constexpr (PL == 2) {
                jr[s][PL - 1][0] = ld16(jsrc_lo + o);
                jr[s][PL - 1][1] = ld16(jsrc_lo + o + 1024);
            }
        }
    };
    auto load_x = [&](uint4 (&d)[MBW][PL][2], int kc) {
        const int64_t o = chunk_at(kc) * XCH;
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) {
            d[mb][0][0] = ld16(xsrc + o + mb * FRAG_BYTES);
            d[mb][0][1] = ld16(xsrc + o + mb * FRAG_BYTES + 1024);
            if constexpr (PL == 2) {
                d[mb][PL - 1][0] = ld16(xsrc_lo + o + mb * FRAG_BYTES);
                d[mb][PL - 1][1] = ld16(xsrc_lo + o + mb * FRAG_BYTES + 1024);
            }
        }
    };

    // nkc is a multiple of PD (the host pads N accordingly). Every chunk
    // issues the same loads (the last PD chunks re-read their own chunk
    // instead of prefetching past the end), so the memory counters the
    // compiler waits on are exact and the loop body has no branches; the
    // prologue issues its loads in the loop's order, J then operand per chunk.
#pragma unroll
    for (int s = 0; s < PD; ++s) {
        load_j(s, s);
        __builtin_amdgcn_sched_barrier(0);
        load_x(xr[s], s);
        __builtin_amdgcn_sched_barrier(0);
    }

#pragma unroll 1
    for (int kc0 = 0; kc0 < nkc; kc0 += PD) {
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            const int kc = kc0 + s;
            const int kn = (kc + PD < nkc) ? kc + PD : kc;
            uint8_t *slot = lds + (kc & 1) * SLOT;
            // publish this wave's J fragment of chunk kc (bit-packed J is
            // expanded to e4m3 bytes here); slot (kc & 1) was last read in
            // chunk kc - 2, which every wave finished before the barrier of
            // chunk kc - 1
            if constexpr (JPK) {
                Frag32 f;
                if constexpr (is_fp4<PATH>) f = unpack_pm1_fp4(jw[s]);
                else f = unpack_pm1(jw[s]);
                uint8_t *dst = slot + w * FRAG_BYTES + l16;
                *reinterpret_cast<uint4 *>(dst) = f.lo;
                *reinterpret_cast<uint4 *>(dst + 1024) = f.hi;
            } else if constexpr (CG == 2) {
                uint8_t *dst = slot + (cg * RBT + w) * FRAG_BYTES + l16;
                *reinterpret_cast<uint4 *>(dst) = jr[s][0][0];
                *reinterpret_cast<uint4 *>(dst + 1024) = jr[s][0][1];
            } else {
#pragma unroll
                for (int pl = 0; pl < PL; ++pl) {
                    uint8_t *dst = slot + (pl * RBT + w) * FRAG_BYTES + l16;
                    *reinterpret_cast<uint4 *>(dst) = jr[s][pl][0];
                    *reinterpret_cast<uint4 *>(dst + 1024) = jr[s][pl][1];
                }
            }
            load_j(s, kn);
            __syncthreads();
            // J fragments of the 4 row blocks, two in registers at a time
            Frag32 bjb[2][PL];
            auto read_j = [&](Frag32 (&d)[PL], int p) {
#pragma unroll
                for (int pl = 0; pl < PL; ++pl) {
                    d[pl].lo = *reinterpret_cast<const uint4 *>(slot + (pl * RBT + p) * FRAG_BYTES + l16);
                    d[pl].hi = *reinterpret_cast<const uint4 *>(slot + (pl * RBT + p) * FRAG_BYTES + 1024 + l16);
                }
            };
            read_j(bjb[0], 0);
#pragma unroll
            for (int p = 0; p < RBT; ++p) {
                if (p + 1 < RBT) read_j(bjb[(p + 1) & 1], p + 1);
                const Frag32 &bj = bjb[p & 1][0], &bj2 = bjb[p & 1][PL - 1];
                // term-major order: consecutive MFMAs go to different blocks
                static_for<0, NT>([&](auto tc) {
                    constexpr int T = decltype(tc)::value;
#pragma unroll
                    for (int mb = 0; mb < MBW; ++mb) {
                        const Frag32 ax{xr[s][mb][0][0], xr[s][mb][0][1]};
                        const Frag32 ax2{xr[s][mb][PL - 1][0], xr[s][mb][PL - 1][1]};
                        mma_term<PATH, T>(acc[mb][p], ax, bj, ax2, bj2);
                    }
                });
                // keeps the fragment reads two row blocks deep (register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
            load_x(xr[s], kn);
        }
    }

    dense_epilogue<PATH, MBW, EPI>(a, acc, nt, mchunk, lds, w);
}

template <int PATH, int MBW, int EPI>
__global__ __launch_bounds__(DENSE_THREADS) void k_dense_step(const DenseStepArgs a) {
    dense_step_body<PATH, MBW, EPI>(a, blockIdx.x, blockIdx.y);
}

// The same step with two column groups per workgroup (two J planes, each
// staged by one group): grid (Np / DENSE_TN, Cg / (128 * MBW)).
template <int PATH, int MBW, int EPI>
__global__ __launch_bounds__(2 * DENSE_THREADS) void k_dense_step_cg2(const DenseStepArgs a) {
    dense_step_body<PATH, MBW, EPI, 2>(a, blockIdx.x, blockIdx.y);
}

// K chunks in flight per wave in the split-K kernel (fp8 and fp4 alike;
// measured: four fp8 chunks in flight 3% slower, four fp4 chunks 4% slower)
constexpr int SK_DEPTH = 2;

// Split-K step for exact contractions: a 128-spin tile (8 row blocks) x
// 64*MBW columns, 8 waves; waves 0-3 sum the first half of K and waves 4-7
// the second, each wave owning MBW m-blocks and all 8 row blocks, so every
// operand fragment feeds 8 row blocks. The halves are added through LDS
// (integer-valued sums: the order does not change the result), then wave
// (h, w) runs the update epilogue of the 64-spin half h. J is staged through
// LDS two K chunks at a time (four slots per half), one barrier per pair.
template <int PATH, int MBW, int EPI>
__global__ __launch_bounds__(2 * DENSE_THREADS) void k_dense_step_sk(const DenseStepArgs a) {
    static_assert(path_packed(Path(PATH)), "split-K kernel: bit-packed exact paths only");
    constexpr int PD = SK_DEPTH;
    constexpr int NT = Terms<PATH>::n;
    constexpr int RBG = DENSE_TN / 16;            // row blocks per 64-spin J group
    constexpr int RB = 2 * RBG;                   // row blocks per tile
    constexpr int SLOT = RB * FRAG_BYTES;         // expanded J of one K chunk
    constexpr int TS = DENSE_TN + 4;
    constexpr int TBYTES = 8 * 16 * TS * 4;
    constexpr int RBYTES = 2 * 4 * MBW * RBG * 64 * 16;
    constexpr int JB = 8 * SLOT;                  // 4 slots per K half: one barrier per 2 chunks
    static_assert(PD % 2 == 0, "chunks are staged in pairs");
    constexpr int LDS_BYTES = JB > TBYTES ? (JB > RBYTES ? JB : RBYTES) : (TBYTES > RBYTES ? TBYTES : RBYTES);
    __shared__ __align__(16) uint8_t lds[LDS_BYTES];

    const int nt2 = blockIdx.x, mchunk = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = wv >> 2, w = wv & 3;
    const int nkc = a.nkc, nkh = nkc / 2;
    const int l16 = lane * 16;
    constexpr int JFRAG = pk_frag_bytes(Path(PATH));
    using JWord = std::conditional_t<is_fp4<PATH>, uint2, uint32_t>;
    constexpr int JCH = RBG * JFRAG;
    constexpr int XCH = MBW * FRAG_BYTES;
    // this wave stages row blocks 2w and 2w+1 of the tile (J group 2*nt2 + w/2)
    const int64_t jgrp = (int64_t)(2 * nt2 + (w >> 1)) * nkc * JCH + ((2 * w) & 3) * JFRAG + lane * (int)sizeof(JWord);
    const int64_t xgrp = (int64_t)(mchunk * 4 + w) * nkc * XCH + l16;
    const uint8_t *jsrc = a.J + jgrp;
    const uint8_t *xsrc = a.g + xgrp;

    JWord jw[PD][2];
    uint4 xr[PD][MBW][2];
    f4 acc[MBW][RB];
#pragma unroll
    for (int i = 0; i < MBW; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[i][j] = f4{0, 0, 0, 0};

    const int rev = a.reverse;
    auto chunk_at = [&](int j) -> int64_t { const int kc = h * nkh + j; return rev ? nkc - 1 - kc : kc; };
    auto load_j = [&](int s, int j) {
        const int64_t o = chunk_at(j) * JCH;
        jw[s][0] = *reinterpret_cast<const JWord *>(jsrc + o);
        jw[s][1] = *reinterpret_cast<const JWord *>(jsrc + o + JFRAG);
    };
    auto load_x = [&](uint4 (&d)[MBW][2], int j) {
        const int64_t o = chunk_at(j) * XCH;
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) {
            d[mb][0] = ld16(xsrc + o + mb * FRAG_BYTES);
            d[mb][1] = ld16(xsrc + o + mb * FRAG_BYTES + 1024);
        }
    };
#pragma unroll
    for (int s = 0; s < PD; ++s) {
        load_j(s, s);
        __builtin_amdgcn_sched_barrier(0);
        load_x(xr[s], s);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll 1
    for (int j0 = 0; j0 < nkh; j0 += PD) {
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            const int j = j0 + s;
            const int jn = (j + PD < nkh) ? j + PD : j;
            uint8_t *slot = lds + (h * 4 + (j & 3)) * SLOT;
            // chunks j and j + 1 are staged together (slots j % 4 and
            // (j + 1) % 4 were last read for chunks j - 4 and j - 3, which
            // every wave finished before the barrier of chunk pair j - 2)
            if (s % 2 == 0) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        Frag32 f;
                        if constexpr (is_fp4<PATH>) f = unpack_pm1_fp4(jw[s + q][e]);
                        else f = unpack_pm1(jw[s + q][e]);
                        uint8_t *dst = lds + (h * 4 + ((j + q) & 3)) * SLOT + (2 * w + e) * FRAG_BYTES + l16;
                        *reinterpret_cast<uint4 *>(dst) = f.lo;
                        *reinterpret_cast<uint4 *>(dst + 1024) = f.hi;
                    }
                const int jn1 = (j + 1 + PD < nkh) ? j + 1 + PD : j + 1;
                load_j(s, jn);
                load_j(s + 1, jn1);
                __syncthreads();
            }
            Frag32 bjb[2];
            auto read_j = [&](Frag32 &d, int p) {
                d.lo = *reinterpret_cast<const uint4 *>(slot + p * FRAG_BYTES + l16);
                d.hi = *reinterpret_cast<const uint4 *>(slot + p * FRAG_BYTES + 1024 + l16);
            };
            read_j(bjb[0], 0);
#pragma unroll
            for (int p = 0; p < RB; ++p) {
                if (p + 1 < RB) read_j(bjb[(p + 1) & 1], p + 1);
                const Frag32 &bj = bjb[p & 1];
                static_for<0, NT>([&](auto tc) {
                    constexpr int T = decltype(tc)::value;
#pragma unroll
                    for (int mb = 0; mb < MBW; ++mb) {
                        const Frag32 ax{xr[s][mb][0], xr[s][mb][1]};
                        mma_term<PATH, T>(acc[mb][p], ax, bj, ax, bj);
                    }
                });
                __builtin_amdgcn_sched_barrier(0);
            }
            load_x(xr[s], jn);
        }
    }
    // add the two K halves: wave (h, w) keeps row blocks [4h, 4h + 4)
    __syncthreads();
    f4 *red = reinterpret_cast<f4 *>(lds);
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
        for (int p = 0; p < RBG; ++p)
            red[(((h * 4 + w) * MBW + mb) * RBG + p) * 64 + lane] = h == 0 ? acc[mb][RBG + p] : acc[mb][p];
    __syncthreads();
    f4 mine[MBW][RBG];
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
        for (int p = 0; p < RBG; ++p) {
            const f4 o = red[((((1 - h) * 4 + w) * MBW + mb) * RBG + p) * 64 + lane];
            const f4 m = h == 0 ? acc[mb][p] : acc[mb][RBG + p];
            mine[mb][p] = f4{m[0] + o[0], m[1] + o[1], m[2] + o[2], m[3] + o[3]};
        }
    dense_epilogue<PATH, MBW, EPI>(a, mine, 2 * nt2 + h, mchunk, lds, w);
}

// Grouped step of every dense instance of one serving group (same path and
// m-blocks per wave): a grid-stride loop over the tiles of all tasks (task q
// owns virtual blocks [first, first + nblocks), nchunk spin tiles per column
// chunk), each running exactly the workgroup of the standalone kernel for the
// task's step n = n_base + offset; tasks past their last step skip.
// J in the contraction precision, fragment-tiled (groups of DENSE_TN/16 row
// blocks), from the zero-padded row-major float64 copy: one thread per 4
// consecutive K elements of a row. e4m3 for ternary J, int8 for integer J
// with |J| <= 127 (both validated on the host), float32 round-to-nearest, or
// bf16 hi = rne(J), lo = rne(J - hi) in float64.
template <int PATH>
__global__ __launch_bounds__(256) void k_convert_j(const double *__restrict__ J64, int Np, int nkc,
                                                   uint8_t *__restrict__ Jd, uint8_t *__restrict__ Jd_lo) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nq = (int64_t)Np * (Np / 4);
    if (q >= nq) return;
    const int row = (int)(q / (Np / 4)), k4 = (int)(q % (Np / 4)) * 4;
    const double *src = J64 + (int64_t)row * Np + k4;
    const int64_t o = op_offset<PATH>(row, k4, nkc, DENSE_TN / 16);
    if constexpr (PATH == PATH_F32) {
        *reinterpret_cast<float4 *>(Jd + o) = make_float4((float)src[0], (float)src[1], (float)src[2], (float)src[3]);
    } else if constexpr (PATH == PATH_FP8) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t b = src[e] > 0.0 ? FP8_P1 : (src[e] < 0.0 ? FP8_M1 : 0u);
            w |= b << (8 * e);
        }
        *reinterpret_cast<uint32_t *>(Jd + o) = w;
    } else if constexpr (PATH == PATH_I8) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= ((uint32_t)(int32_t)src[e] & 0xFFu) << (8 * e);
        *reinterpret_cast<uint32_t *>(Jd + o) = w;
    } else if constexpr (PATH == PATH_FP4) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= (src[e] > 0.0 ? FP4_P1 : (src[e] < 0.0 ? FP4_M1 : 0u)) << (4 * e);
        *reinterpret_cast<uint16_t *>(Jd + o) = (uint16_t)w;
    } else {
        uint16_t hi[4], lo[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            hi[e] = bf16_rne((float)src[e]);
            lo[e] = bf16_rne((float)(src[e] - (double)bf16_to_f32(hi[e])));
        }
        *reinterpret_cast<uint2 *>(Jd + o) = make_uint2(hi[0] | ((uint32_t)hi[1] << 16), hi[2] | ((uint32_t)hi[3] << 16));
        *reinterpret_cast<uint2 *>(Jd_lo + o) = make_uint2(lo[0] | ((uint32_t)lo[1] << 16), lo[2] | ((uint32_t)lo[3] << 16));
    }
}

// Bit-packed +-1 J (layouts of unpack_pm1 / unpack_pm1_fp4), fragment-tiled
// like the byte copy (groups of DENSE_TN/16 row blocks): one thread per
// (fragment, lane, dword), consecutive threads write consecutive dwords. A bit
// is set where J_ij < 0; the diagonal and the padding read 0 and so hold +1
// (the step's epilogue removes both). `neg(i, j)` tells whether J_ij < 0 for
// i, j < Np: from the zero-padded float64 copy, or from row-major sign bits.
template <bool FP4, class Neg>
__device__ __forceinline__ void convert_j_pk(int Np, int nkc, uint32_t *__restrict__ Jd, Neg neg) {
    constexpr int RBT = DENSE_TN / 16, DW = FP4 ? 2 : 1;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)(Np / 16) * nkc * 64 * DW) return;
    const int d = (int)(q % DW), lane = (int)((q / DW) & 63);
    const int64_t frag = q / DW / 64;
    const int w = (int)(frag % RBT);
    const int64_t t = frag / RBT;
    const int kc = (int)(t % nkc), rb = (int)(t / nkc) * RBT + w;
    const int g = lane >> 4;
    const int i = 16 * rb + (lane & 15);
    uint32_t bits = 0;
    if constexpr (FP4) {
        // half d: K = 256 kc + 64 g + 32 d + 8 k + i for nibble i of dword k
        const int j0 = 256 * kc + 64 * g + 32 * d;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (neg(i, j0 + 8 * k + e)) bits |= 1u << (4 * e + k);
    } else {
        // byte b = 4 k + e of the lane's 32: K = 128 kc + 32 g + 16 (b / 16) + b % 16
        const int j0 = 128 * kc + 32 * g;
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int bb = 4 * k + e;
                if (neg(i, j0 + 16 * (bb >> 4) + (bb & 15))) bits |= 1u << (8 * e + k);
            }
    }
    Jd[q] = bits;
}

template <bool FP4>
__global__ __launch_bounds__(256) void k_convert_j_pk(const double *__restrict__ J64, int Np, int nkc,
                                                     uint32_t *__restrict__ Jd) {
    convert_j_pk<FP4>(Np, nkc, Jd, [&](int i, int j) { return J64[(int64_t)i * Np + j] < 0.0; });
}

// From row-major sign bits of an N x N matrix (bit j % 32 of word
// i * words + j / 32 set where J_ij < 0); rows and columns past N read +1.
template <bool FP4>
__global__ __launch_bounds__(256) void k_convert_j_pk_bits(const uint32_t *__restrict__ sb, int N, int words, int Np,
                                                          int nkc, uint32_t *__restrict__ Jd) {
    convert_j_pk<FP4>(Np, nkc, Jd, [&](int i, int j) {
        return i < N && j < N && ((sb[(int64_t)i * words + (j >> 5)] >> (j & 31)) & 1u) != 0u;
    });
}

template <int PATH, int MBW>
__global__ __launch_bounds__(DENSE_THREADS) void k_group_dense(const GroupHeader *__restrict__ hdr,
                                                               const GroupTask *__restrict__ tasks, int offset) {
    const int ntask = hdr->ntask, total = hdr->total_blocks;
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        int q = 0;
        while (q + 1 < ntask && tasks[q + 1].first_block <= vb) ++q;
        const GroupTask &t = tasks[q];
        const int n = t.n_base + offset;
        if (n >= t.n_end) continue;
        const int in = n & 1, lt = vb - t.first_block;
        DenseStepArgs a;
        a.N = t.N;
        a.Np = t.ld;
        a.R = t.R;
        a.C = t.C;
        a.nkc = t.nkc;
        a.reverse = in;
        a.J = static_cast<const uint8_t *>(t.J);
        a.J_lo = static_cast<const uint8_t *>(t.J_lo);
        a.g = static_cast<const uint8_t *>(t.g[in]);
        a.g_lo = static_cast<const uint8_t *>(t.g_lo[in]);
        a.g_next = static_cast<uint8_t *>(t.g[1 - in]);
        a.g_next_lo = static_cast<uint8_t *>(t.g_lo[1 - in]);
        a.h = t.h;
        a.x_in = t.x[in];
        a.x_out = t.x[1 - in];
        a.y = t.y;
        a.phi = nullptr;
        a.jp = t.jp + n;
        a.jp_stride = t.S;
        a.k.kA = t.coefA[n];
        a.k.kB = t.kB;
        a.k.dt = t.dt;
        a.k.kD = t.kD;
        a.k.delta_next = t.delta[n + 1];
        a.fmode = t.fmode;
        dense_step_body<PATH, MBW, EPI_UPDATE>(a, lt % t.nchunk, lt / t.nchunk);
    }
}

// Operand f(X) from the state: one thread per 4 consecutive spins of column c.
template <int PATH>
__global__ __launch_bounds__(256) void k_dense_operand(int Np, int nkc, int mbw, const float *__restrict__ x, void *g,
                                                       void *g_lo, float delta, int fmode) {
    const int c = blockIdx.y;
    const int i4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i4 >= Np) return;
    const float4 v = *reinterpret_cast<const float4 *>(x + (int64_t)c * Np + i4);
    const float4 f = make_float4(f_value(fmode, v.x, delta), f_value(fmode, v.y, delta),
                                 f_value(fmode, v.z, delta), f_value(fmode, v.w, delta));
    store_operand<PATH>(g, g_lo, op_offset<PATH>(c, i4, nkc, mbw), f, fmode);
}

// Readout operand s = sign(x) with sign(0) = +1 (the energy convention of
// Eq. 2 at the corners), 0 for padded spins i >= N: the dense contraction of
// it gives J s exactly (integer J in fp8 / int8, |J s| < 2^24).
template <int PATH>
__global__ __launch_bounds__(256) void k_readout_operand(int N, int Np, int nkc, int mbw, const float *__restrict__ x,
                                                         void *g) {
    const int c = blockIdx.y;
    const int i4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i4 >= Np) return;
    const float4 v = *reinterpret_cast<const float4 *>(x + (int64_t)c * Np + i4);
    auto s = [N](float xv, int i) { return i < N ? (xv >= 0.0f ? 1.0f : -1.0f) : 0.0f; };
    const float4 f = make_float4(s(v.x, i4), s(v.y, i4 + 1), s(v.z, i4 + 2), s(v.w, i4 + 3));
    store_operand<PATH>(g, nullptr, op_offset<PATH>(c, i4, nkc, mbw), f, 0);
}

template <int PATH, int EPI>
hipError_t launch_step_mbw(int mbw, dim3 grid, const DenseStepArgs &a, hipStream_t st) {
    // 128-column tile of a bit-packed path: the split-K form when both K
    // halves fill the prefetch pipeline (same fields, integer-valued sums)
    if constexpr (path_packed(Path(PATH))) {
        if (mbw == 2 && a.nkc % (2 * SK_DEPTH) == 0 && grid.x % 2 == 0) {
            hipLaunchKernelGGL((k_dense_step_sk<PATH, 2, EPI>), dim3(grid.x / 2, grid.y), dim3(2 * DENSE_THREADS), 0, st, a);
            return hipGetLastError();
        }
    }
    // two J planes: two column groups per workgroup read each J fragment once
    // for 256 columns (half the J traffic of two 128-column workgroups)
    if constexpr (Pipe<PATH>::planes == 2) {
        if (mbw == 2 && grid.y % 2 == 0) {
            hipLaunchKernelGGL((k_dense_step_cg2<PATH, 2, EPI>), dim3(grid.x, grid.y / 2), dim3(2 * DENSE_THREADS), 0, st,
                               a);
            return hipGetLastError();
        }
    }
    switch (mbw) {
        case 1: hipLaunchKernelGGL((k_dense_step<PATH, 1, EPI>), grid, dim3(DENSE_THREADS), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_dense_step<PATH, 2, EPI>), grid, dim3(DENSE_THREADS), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_dense_step<PATH, 4, EPI>), grid, dim3(DENSE_THREADS), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PATH>
hipError_t launch_step_path(DenseEpilogue epi, int mbw, dim3 grid, const DenseStepArgs &a, hipStream_t st) {
    return epi == EPI_UPDATE ? launch_step_mbw<PATH, EPI_UPDATE>(mbw, grid, a, st)
                             : launch_step_mbw<PATH, EPI_FIELDS>(mbw, grid, a, st);
}

}  // namespace

hipError_t launch_gemm_f64(const double *A, const double *B, double *out, int Np, int Cp, int splits,
                           hipStream_t st) {
    const int64_t kbytes = (int64_t)Np * 8;
    if (Np % GEMM_BN || Cp % GEMM_BM || splits < 1 || kbytes % ((int64_t)splits * GEMM_KB))
        return hipErrorInvalidValue;
    const int kchunk = (int)(kbytes / splits);
    dim3 grid(Np / GEMM_BN, Cp / GEMM_BM, splits), block(GEMM_THREADS);
    hipLaunchKernelGGL(k_gemm_f64, grid, block, 0, st, reinterpret_cast<const uint8_t *>(A),
                       reinterpret_cast<const uint8_t *>(B), out, Np, Cp, kchunk);
    return hipGetLastError();
}

hipError_t launch_dense_step(Path path, DenseEpilogue epi, int mbw, int Cg, const DenseStepArgs &a,
                             hipStream_t st) {
    const int tm = 64 * mbw;
    if (a.Np % DENSE_TN || Cg % tm || a.C > Cg || a.Np % path_kpc(path) || a.nkc != dense_nkc(path, a.Np) ||
        a.nkc % dense_depth(path))
        return hipErrorInvalidValue;
    const dim3 grid(a.Np / DENSE_TN, Cg / tm);
    switch (path) {
        case PATH_F32: return launch_step_path<PATH_F32>(epi, mbw, grid, a, st);
        case PATH_FP8: return launch_step_path<PATH_FP8>(epi, mbw, grid, a, st);
        case PATH_BF16X3: return launch_step_path<PATH_BF16X3>(epi, mbw, grid, a, st);
        case PATH_I8: return launch_step_path<PATH_I8>(epi, mbw, grid, a, st);
        case PATH_FP8PK: return launch_step_path<PATH_FP8PK>(epi, mbw, grid, a, st);
        case PATH_FP4: return launch_step_path<PATH_FP4>(epi, mbw, grid, a, st);
        case PATH_FP4PK: return launch_step_path<PATH_FP4PK>(epi, mbw, grid, a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_convert_j_bits(Path path, const uint32_t *sign_bits, int N, int Np, int nkc, void *Jd,
                                 hipStream_t st) {
    if (!path_packed(path) || Np % 128 || Np % path_kpc(path) || nkc != dense_nkc(path, Np) || N > Np)
        return hipErrorInvalidValue;
    const bool fp4 = path_fp4(path);
    const int words = (N + 31) / 32;
    const int64_t nq = (int64_t)(Np / 16) * nkc * 64 * (fp4 ? 2 : 1);
    const dim3 grid((unsigned)((nq + 255) / 256));
    if (fp4)
        hipLaunchKernelGGL(k_convert_j_pk_bits<true>, grid, dim3(256), 0, st, sign_bits, N, words, Np, nkc,
                           static_cast<uint32_t *>(Jd));
    else
        hipLaunchKernelGGL(k_convert_j_pk_bits<false>, grid, dim3(256), 0, st, sign_bits, N, words, Np, nkc,
                           static_cast<uint32_t *>(Jd));
    return hipGetLastError();
}

hipError_t launch_convert_j(Path path, const double *J64, int Np, int nkc, void *Jd, void *Jd_lo, hipStream_t st) {
    if (Np % 128 || Np % path_kpc(path) || nkc != dense_nkc(path, Np)) return hipErrorInvalidValue;
    if (path_packed(path)) {
        const bool fp4 = path_fp4(path);
        const int64_t nq = (int64_t)(Np / 16) * nkc * 64 * (fp4 ? 2 : 1);
        const dim3 grid((unsigned)((nq + 255) / 256));
        if (fp4) hipLaunchKernelGGL(k_convert_j_pk<true>, grid, dim3(256), 0, st, J64, Np, nkc, static_cast<uint32_t *>(Jd));
        else hipLaunchKernelGGL(k_convert_j_pk<false>, grid, dim3(256), 0, st, J64, Np, nkc, static_cast<uint32_t *>(Jd));
        return hipGetLastError();
    }
    const int64_t nq = (int64_t)Np * (Np / 4);
    const dim3 grid((unsigned)((nq + 255) / 256)), block(256);
    uint8_t *d = static_cast<uint8_t *>(Jd), *dl = static_cast<uint8_t *>(Jd_lo);
    switch (path) {
        case PATH_F32: hipLaunchKernelGGL(k_convert_j<PATH_F32>, grid, block, 0, st, J64, Np, nkc, d, dl); break;
        case PATH_FP8: hipLaunchKernelGGL(k_convert_j<PATH_FP8>, grid, block, 0, st, J64, Np, nkc, d, dl); break;
        case PATH_BF16X3: hipLaunchKernelGGL(k_convert_j<PATH_BF16X3>, grid, block, 0, st, J64, Np, nkc, d, dl); break;
        case PATH_I8: hipLaunchKernelGGL(k_convert_j<PATH_I8>, grid, block, 0, st, J64, Np, nkc, d, dl); break;
        case PATH_FP4: hipLaunchKernelGGL(k_convert_j<PATH_FP4>, grid, block, 0, st, J64, Np, nkc, d, dl); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_group_dense(Path path, int mbw, const GroupHeader *hdr, const GroupTask *tasks, int grid,
                              int offset, hipStream_t st) {
    if (grid < 1) return hipErrorInvalidValue;
#define SBQA_GD(P, M) hipLaunchKernelGGL((k_group_dense<P, M>), dim3(grid), dim3(DENSE_THREADS), 0, st, hdr, tasks, offset)
#define SBQA_GD_PATH(P)                 \
    switch (mbw) {                      \
        case 1: SBQA_GD(P, 1); break;   \
        case 2: SBQA_GD(P, 2); break;   \
        case 4: SBQA_GD(P, 4); break;   \
        default: return hipErrorInvalidValue; \
    }
    switch (path) {
        case PATH_F32: SBQA_GD_PATH(PATH_F32); break;
        case PATH_FP8: SBQA_GD_PATH(PATH_FP8); break;
        case PATH_BF16X3: SBQA_GD_PATH(PATH_BF16X3); break;
        case PATH_I8: SBQA_GD_PATH(PATH_I8); break;
        case PATH_FP8PK: SBQA_GD_PATH(PATH_FP8PK); break;
        case PATH_FP4: SBQA_GD_PATH(PATH_FP4); break;
        case PATH_FP4PK: SBQA_GD_PATH(PATH_FP4PK); break;
        default: return hipErrorInvalidValue;
    }
#undef SBQA_GD_PATH
#undef SBQA_GD
    return hipGetLastError();
}

hipError_t launch_dense_operand(Path path, int fmode, int N, int Np, int C, int nkc, int mbw, const float *x, void *g,
                                void *g_lo, float delta, hipStream_t st) {
    (void)N;
    dim3 grid((Np / 4 + 255) / 256, C), block(256);
    switch (path) {
        case PATH_F32: hipLaunchKernelGGL(k_dense_operand<PATH_F32>, grid, block, 0, st, Np, nkc, mbw, x, g, g_lo, delta, fmode); break;
        case PATH_FP8: hipLaunchKernelGGL(k_dense_operand<PATH_FP8>, grid, block, 0, st, Np, nkc, mbw, x, g, g_lo, delta, fmode); break;
        case PATH_BF16X3: hipLaunchKernelGGL(k_dense_operand<PATH_BF16X3>, grid, block, 0, st, Np, nkc, mbw, x, g, g_lo, delta, fmode); break;
        case PATH_I8: hipLaunchKernelGGL(k_dense_operand<PATH_I8>, grid, block, 0, st, Np, nkc, mbw, x, g, g_lo, delta, fmode); break;
        case PATH_FP8PK: hipLaunchKernelGGL(k_dense_operand<PATH_FP8>, grid, block, 0, st, Np, nkc, mbw, x, g, g_lo, delta, fmode); break;
        case PATH_FP4:
        case PATH_FP4PK: hipLaunchKernelGGL(k_dense_operand<PATH_FP4>, grid, block, 0, st, Np, nkc, mbw, x, g, g_lo, delta, fmode); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sbqa

namespace sbqa {

hipError_t launch_readout_operand(Path path, int N, int Np, int C, int nkc, int mbw, const float *x, void *g,
                                  hipStream_t st) {
    dim3 grid((Np / 4 + 255) / 256, C), block(256);
    switch (path) {
        case PATH_FP8:
        case PATH_FP8PK: hipLaunchKernelGGL(k_readout_operand<PATH_FP8>, grid, block, 0, st, N, Np, nkc, mbw, x, g); break;
        case PATH_I8: hipLaunchKernelGGL(k_readout_operand<PATH_I8>, grid, block, 0, st, N, Np, nkc, mbw, x, g); break;
        case PATH_FP4:
        case PATH_FP4PK: hipLaunchKernelGGL(k_readout_operand<PATH_FP4>, grid, block, 0, st, N, Np, nkc, mbw, x, g); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sbqa
