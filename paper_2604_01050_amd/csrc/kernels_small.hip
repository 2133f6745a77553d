// Resident loop for small dense instances (gfx950): one workgroup per run
// keeps J (float32) and the positions and operand of its R replicas in LDS and
// the velocities in registers, and advances K steps of Eqs. 6-7 per launch,
// so a small all-to-all instance costs one launch per K steps instead of one
// per step. Fields are summed in a fixed order over j (four interleaved
// partial sums), so integer couplings with a ternary or sign operand give
// exactly the fields of the MFMA path.
#include "sbqa_internal.h"

namespace sbqa {
namespace {

constexpr int SM_THREADS = 512;   // two waves per SIMD: 1.50 against 1.99 us per step at N = 64, R = 8
constexpr int SM_EPT = SMALL_MAX_ELEMS / SM_THREADS;  // replica-spin elements per thread

__device__ __forceinline__ float f_small(int fmode, float x, float delta) {
    if (fmode == 2) return x;                       // bSB
    const float d = (fmode == 1) ? 0.0f : delta;    // dSB: sign(0) = 0
    if (fabsf(x) <= d) return 0.0f;
    return x > 0.0f ? 1.0f : -1.0f;
}

#pragma clang fp contract(off)
__global__ __launch_bounds__(SM_THREADS) void k_dense_small(const SmallArgs a) {
    extern __shared__ float sm[];
    const int N = a.N, R = a.R, NS = N + 1;      // odd J row stride: conflict-free column walks
    float *Js = sm;                               // [N][N+1]
    float *xs = Js + N * NS;                      // [R][N] positions of this run
    float *fs = xs + R * N;                       // [R][N] operand f(x)
    const int run = blockIdx.x, tid = threadIdx.x, E = R * N;
    for (int e = tid; e < N * N; e += SM_THREADS) Js[(e / N) * NS + e % N] = a.J[e];

    // this thread's elements e = tid + q*SM_THREADS: replica k = e / N, spin i = e % N
    float yv[SM_EPT], hv[SM_EPT];
    int ek[SM_EPT], ei[SM_EPT];
#pragma unroll
    for (int q = 0; q < SM_EPT; ++q) {
        const int e = tid + q * SM_THREADS;
        ek[q] = e / N;
        ei[q] = e - ek[q] * N;
        if (e < E) {
            const int64_t o = (int64_t)(run * R + ek[q]) * a.Np + ei[q];
            const float x = a.x[o];
            xs[e] = x;
            fs[e] = f_small(a.fmode, x, a.delta[a.n0]);
            yv[q] = a.y[o];
            hv[q] = a.h[ei[q]];
        }
    }
    __syncthreads();

    for (int n = a.n0; n < a.n0 + a.K; ++n) {
        const float kA = a.coefA[n], dnext = a.delta[n + 1], jpr = a.jp[(int64_t)run * a.S + n];
        float xn[SM_EPT];
#pragma unroll
        for (int q = 0; q < SM_EPT; ++q) {
            const int e = tid + q * SM_THREADS;
            if (e >= E) continue;
            const int k = ek[q], i = ei[q];
            const float *jrow = Js + i * NS, *frow = fs + k * N;
            // four interleaved partial sums over j = 4m + u, then (s0 + s1) +
            // (s2 + s3): a fixed order with four independent FMA chains
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
            int j = 0;
            for (; j + 3 < N; j += 4) {
                s0 = fmaf(jrow[j], frow[j], s0);
                s1 = fmaf(jrow[j + 1], frow[j + 1], s1);
                s2 = fmaf(jrow[j + 2], frow[j + 2], s2);
                s3 = fmaf(jrow[j + 3], frow[j + 3], s3);
            }
            for (; j < N; ++j) s0 = fmaf(jrow[j], frow[j], s0);
            const float phi = (s0 + s1) + (s2 + s3);
            const int kl = (k == 0) ? R - 1 : k - 1, kr = (k == R - 1) ? 0 : k + 1;
            const float x = xs[e], xl = xs[kl * N + i], xr = xs[kr * N + i];
            const float force = (-kA * x + a.kB * (phi + hv[q])) + jpr * (xl + xr);
            float yn = yv[q] + a.dt * force;
            float xv = x + a.kD * yn;
            if (fabsf(xv) > 1.0f) {
                xv = xv > 0.0f ? 1.0f : -1.0f;
                yn = 0.0f;
            }
            yv[q] = yn;
            xn[q] = xv;
        }
        __syncthreads();   // every read of step n's positions and operand is done
#pragma unroll
        for (int q = 0; q < SM_EPT; ++q) {
            const int e = tid + q * SM_THREADS;
            if (e >= E) continue;
            xs[e] = xn[q];
            fs[e] = f_small(a.fmode, xn[q], dnext);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < SM_EPT; ++q) {
        const int e = tid + q * SM_THREADS;
        if (e >= E) continue;
        const int64_t o = (int64_t)(run * R + ek[q]) * a.Np + ei[q];
        a.x[o] = xs[e];
        a.y[o] = yv[q];
    }
}
#pragma clang fp contract(on)

}  // namespace

size_t small_lds_bytes(int N, int R) { return sizeof(float) * ((size_t)N * (N + 1) + 2 * (size_t)R * N); }

hipError_t launch_dense_small(const SmallArgs &a, int runs, hipStream_t st) {
    if (a.N < 1 || a.N > SMALL_MAX_N || a.R < 1 || a.R * a.N > SMALL_MAX_ELEMS || a.K < 1 || a.n0 < 0 ||
        a.n0 + a.K > a.S)
        return hipErrorInvalidValue;
    const size_t lds = small_lds_bytes(a.N, a.R);
    hipError_t e = ensure_dyn_lds(reinterpret_cast<const void *>(&k_dense_small), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dense_small, dim3(runs), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}

}  // namespace sbqa
