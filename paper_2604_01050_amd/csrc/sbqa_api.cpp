// Host runtime of the SBQA library: validation, schedules (Eq. 5, Eq. 8 and
// the pump of Sec. II.A), the per-run (beta, alpha) auto-tuning draw of
// Sec. II.B, device buffers, and the step / readout / energy dispatch.
#include "sbqa_ctx.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <tuple>
#include <string>

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>
#include <thread>
#include <vector>

namespace sbqa {

static thread_local std::string g_err;

sbqa_status fail(sbqa_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err.clear(); }
const char *last_error() { return g_err.c_str(); }

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(e_ == hipErrorOutOfMemory ? SBQA_ENOMEM : SBQA_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                     \
    } while (0)

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// splitmix64 (Steele, Lea, Flood 2014): host stream for the (beta, alpha) draws.
static uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double unit_double(uint64_t &s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

// ---------------------------------------------------------------- validation
// One pass over a dense J: diagonal, finiteness, symmetry (64 x 64 tiles of
// the upper triangle against their transposes, so both stay in cache), the
// integral / ternary flags and the sum of squares of the entries. Row blocks
// are scanned in parallel; their sums of squares are added in block order, so
// the result does not depend on the number of threads.
struct DenseScan {
    int bad = 0;              // 1 diagonal, 2 not finite, 3 not symmetric
    int64_t i = 0, j = 0;
    bool integral = true, ternary = true, pm1 = true;
    double ss = 0.0, maxabs = 0.0;
};

static DenseScan scan_dense(const double *A, int64_t N) {
    constexpr int64_t TB = 64;
    const int64_t nb = (N + TB - 1) / TB;
    std::vector<DenseScan> part((size_t)nb);
    auto scan_block = [&](int64_t bi) {
        DenseScan &r = part[(size_t)bi];
        const int64_t i0 = bi * TB, i1 = std::min(N, i0 + TB);
        for (int64_t i = i0; i < i1; ++i) {
            if (A[i * N + i] != 0.0 && !r.bad) { r.bad = 1; r.i = i; r.j = i; }
            double srow = 0.0;
            for (int64_t j = 0; j < N; ++j) {
                const double v = A[i * N + j];
                if (!std::isfinite(v)) {
                    if (!r.bad) { r.bad = 2; r.i = i; r.j = j; }
                    continue;
                }
                if (v != std::floor(v) || std::fabs(v) > 2147483647.0) r.integral = false;
                if (!(v == 0.0 || v == 1.0 || v == -1.0)) r.ternary = false;
                if (j != i && !(v == 1.0 || v == -1.0)) r.pm1 = false;
                r.maxabs = std::max(r.maxabs, std::fabs(v));
                srow += v * v;
            }
            r.ss += srow;
        }
        for (int64_t bj = bi; bj < nb; ++bj) {
            const int64_t j0 = bj * TB, j1 = std::min(N, j0 + TB);
            for (int64_t i = i0; i < i1; ++i)
                for (int64_t j = std::max(j0, i + 1); j < j1; ++j)
                    if (A[i * N + j] != A[j * N + i] && !(std::isnan(A[i * N + j]) && std::isnan(A[j * N + i])) && !r.bad) {
                        r.bad = 3; r.i = i; r.j = j;
                    }
        }
    };
    const int nt = (int)std::min<int64_t>(nb, std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    if (nt <= 1 || N < 512) {
        for (int64_t bi = 0; bi < nb; ++bi) scan_block(bi);
    } else {
        std::vector<std::thread> pool;
        std::atomic<int64_t> next{0};
        for (int t = 0; t < nt; ++t)
            pool.emplace_back([&] {
                for (int64_t bi; (bi = next.fetch_add(1)) < nb;) scan_block(bi);
            });
        for (std::thread &t : pool) t.join();
    }
    DenseScan out;
    for (const DenseScan &r : part) {
        if (r.bad && !out.bad) { out.bad = r.bad; out.i = r.i; out.j = r.j; }
        out.integral = out.integral && r.integral;
        out.ternary = out.ternary && r.ternary;
        out.pm1 = out.pm1 && r.pm1;
        out.maxabs = std::max(out.maxabs, r.maxabs);
        out.ss += r.ss;
    }
    return out;
}

sbqa_status validate_instance(const sbqa_coupling *J, const double *h, int32_t N, int32_t R, int32_t runs,
                              const sbqa_schedule *s, InstanceFacts *facts) {
    if (!J || !s) return fail(SBQA_EINVAL, "J and schedule must be non-NULL");
    if (N < 1 || R < 1 || runs < 1) return fail(SBQA_EINVAL, "N, R and runs must be >= 1 (got %d, %d, %d)", N, R, runs);
    if ((int64_t)R * runs > (1 << 24)) return fail(SBQA_EINVAL, "runs*R too large");
    if (s->steps < 1) return fail(SBQA_EINVAL, "steps must be >= 1");
    if (!(s->dt > 0) || !std::isfinite(s->dt)) return fail(SBQA_EINVAL, "dt must be finite and > 0");
    if (!(s->a0 > 0) || !std::isfinite(s->a0)) return fail(SBQA_EINVAL, "a0 must be finite and > 0");
    if (!std::isfinite(s->c0)) return fail(SBQA_EINVAL, "c0 must be finite");
    if (s->fmode < 0 || s->fmode > 2) return fail(SBQA_EINVAL, "unknown fmode %d", s->fmode);
    if (!std::isfinite(s->delta_max) || s->delta_max < 0) return fail(SBQA_EINVAL, "delta_max must be finite and >= 0");
    if (s->precision < SBQA_PREC_AUTO || s->precision > SBQA_PREC_FP4) return fail(SBQA_EINVAL, "unknown precision %d", s->precision);
    if (s->loop_kernel < 0 || s->loop_kernel > 2) return fail(SBQA_EINVAL, "unknown loop_kernel %d", s->loop_kernel);
    if (s->j_packing < SBQA_JPACK_AUTO || s->j_packing > SBQA_JPACK_BYTES) return fail(SBQA_EINVAL, "unknown j_packing %d", s->j_packing);
    if (s->reorder < SBQA_REORDER_AUTO || s->reorder > SBQA_REORDER_ON) return fail(SBQA_EINVAL, "unknown reorder %d", s->reorder);
    if (s->dense_tile != 0 && s->dense_tile != 64 && s->dense_tile != 128 && s->dense_tile != 256)
        return fail(SBQA_EINVAL, "dense_tile must be 0 (autotuned), 64, 128 or 256 (got %d)", s->dense_tile);
    if (!(s->init_amp >= 0) || !std::isfinite(s->init_amp)) return fail(SBQA_EINVAL, "init_amp must be finite and >= 0");
    switch (s->jp_kind) {
        case SBQA_JP_LINEAR:
            if (!std::isfinite(s->jp_start) || !std::isfinite(s->jp_end)) return fail(SBQA_EINVAL, "jp_start/jp_end must be finite");
            break;
        case SBQA_JP_PAPER:
            if (!(s->gamma0_over_R > 0) || !std::isfinite(s->gamma0_over_R)) return fail(SBQA_EINVAL, "gamma0_over_R must be > 0");
            if (!s->beta && !(s->beta_lo > 0 && s->beta_hi >= s->beta_lo && std::isfinite(s->beta_hi)))
                return fail(SBQA_EINVAL, "need 0 < beta_lo <= beta_hi");
            if (!s->alpha && !(s->alpha_lo > 0 && s->alpha_hi >= s->alpha_lo && std::isfinite(s->alpha_hi)))
                return fail(SBQA_EINVAL, "need 0 < alpha_lo <= alpha_hi");
            if (s->beta)
                for (int r = 0; r < runs; ++r)
                    if (!(s->beta[r] > 0) || !std::isfinite(s->beta[r])) return fail(SBQA_EINVAL, "beta[%d] must be > 0", r);
            if (s->alpha)
                for (int r = 0; r < runs; ++r)
                    if (!(s->alpha[r] > 0) || !std::isfinite(s->alpha[r])) return fail(SBQA_EINVAL, "alpha[%d] must be > 0", r);
            break;
        case SBQA_JP_TABLE:
            if (!s->jp_table) return fail(SBQA_EINVAL, "JP_TABLE needs jp_table");
            for (int64_t q = 0; q < (int64_t)runs * s->steps; ++q)
                if (!std::isfinite(s->jp_table[q])) return fail(SBQA_EINVAL, "jp_table[%lld] not finite", (long long)q);
            break;
        default: return fail(SBQA_EINVAL, "unknown jp_kind %d", s->jp_kind);
    }

    const bool dense = J->dense != nullptr;
    const bool csr = J->row_ptr || J->col || J->val;
    if (dense == csr) return fail(SBQA_EINVAL, "exactly one of J.dense or the CSR arrays must be given");
    bool integral = true, ternary = true;
    double ss = 0.0, maxabs = 0.0;
    auto note = [&](double v) {
        if (v != std::floor(v) || std::fabs(v) > 2147483647.0) integral = false;
        if (!(v == 0.0 || v == 1.0 || v == -1.0)) ternary = false;
        maxabs = std::max(maxabs, std::fabs(v));
    };
    if (dense) {
        if ((int64_t)N * N > (int64_t)1 << 32) return fail(SBQA_EINVAL, "dense N too large");
        const DenseScan d = scan_dense(J->dense, N);
        if (d.bad) {
            switch (d.bad) {
                case 1: return fail(SBQA_EINVAL, "J has a non-zero diagonal at %lld", (long long)d.i);
                case 2: return fail(SBQA_EINVAL, "J[%lld][%lld] is not finite", (long long)d.i, (long long)d.j);
                default: return fail(SBQA_EINVAL, "J is not symmetric at (%lld,%lld)", (long long)d.i, (long long)d.j);
            }
        }
        integral = d.integral;
        ternary = d.ternary;
        facts->pm1 = d.pm1 && N > 1;
        maxabs = d.maxabs;
        ss = d.ss;
        facts->nnz = 0;
    } else {
        if (!J->row_ptr || (J->nnz != 0 && (!J->col || !J->val)))
            return fail(SBQA_EINVAL, "CSR needs row_ptr, and col and val unless nnz is 0");
        const int32_t *rp = J->row_ptr, *cl = J->col;
        const double *vl = J->val;
        if (J->nnz < 0 || rp[0] != 0 || (int64_t)rp[N] != J->nnz) return fail(SBQA_EINVAL, "row_ptr[0] must be 0 and row_ptr[N] == nnz");
        // pass 0: every row's range lies inside [0, nnz] before col or val is read
        for (int32_t i = 0; i < N; ++i)
            if (rp[i + 1] < rp[i] || (int64_t)rp[i + 1] > J->nnz)
                return fail(SBQA_EINVAL, "row_ptr must be non-decreasing within [0, nnz] (row %d)", i);
        // pass 1: structure of every row (so pass 2 may search any row)
        for (int32_t i = 0; i < N; ++i) {
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                if (cl[p] < 0 || cl[p] >= N) return fail(SBQA_EINVAL, "col[%d] = %d out of range", p, cl[p]);
                if (p > rp[i] && cl[p] <= cl[p - 1]) return fail(SBQA_EINVAL, "columns of row %d not strictly ascending", i);
                if (!std::isfinite(vl[p])) return fail(SBQA_EINVAL, "val[%d] not finite", p);
                if (cl[p] == i && vl[p] != 0.0) return fail(SBQA_EINVAL, "J has a non-zero diagonal at %d", i);
            }
        }
        // pass 2: symmetry J_ij == J_ji
        for (int32_t i = 0; i < N; ++i) {
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int32_t j = cl[p];
                const int32_t *b = cl + rp[j], *e = cl + rp[j + 1];
                const int32_t *f = std::lower_bound(b, e, i);
                if (f == e || *f != i || vl[rp[j] + (f - b)] != vl[p])
                    return fail(SBQA_EINVAL, "CSR J is not symmetric at (%d,%d)", i, j);
                note(vl[p]);
                if (j != i) ss += vl[p] * vl[p];
            }
        }
        facts->nnz = J->nnz;
    }
    facts->int8 = integral && maxabs <= 127.0;   // J only: h enters in fp32
    if (J->n3 < 0) return fail(SBQA_EINVAL, "n3 must be >= 0");
    if (J->n3 > 0) {
        if (dense) return fail(SBQA_EINVAL, "three-body terms need CSR two-body couplings (nnz may be 0)");
        if (!J->tri || !J->K) return fail(SBQA_EINVAL, "three-body terms need tri and K");
        if (J->n3 > (int64_t)1 << 28) return fail(SBQA_EINVAL, "too many three-body terms");
        for (int64_t t = 0; t < J->n3; ++t) {
            const int32_t a = J->tri[3 * t], b = J->tri[3 * t + 1], d = J->tri[3 * t + 2];
            if (a < 0 || a >= N || b < 0 || b >= N || d < 0 || d >= N)
                return fail(SBQA_EINVAL, "triple %lld has a spin index out of range", (long long)t);
            if (a == b || a == d || b == d) return fail(SBQA_EINVAL, "triple %lld repeats a spin", (long long)t);
            if (!std::isfinite(J->K[t])) return fail(SBQA_EINVAL, "K[%lld] not finite", (long long)t);
            if (J->K[t] != std::floor(J->K[t])) integral = false;
            ss += 3.0 * J->K[t] * J->K[t];   // field variance of random spins (c0)
        }
    }
    facts->n3 = J->n3 > 0 ? J->n3 : 0;
    if (h)
        for (int32_t i = 0; i < N; ++i) {
            if (!std::isfinite(h[i])) return fail(SBQA_EINVAL, "h[%d] not finite", i);
            if (h[i] != std::floor(h[i])) integral = false;
        }
    facts->dense = dense;
    facts->integral = integral;
    facts->ternary = ternary;
    facts->rms = (N > 1 && ss > 0) ? std::sqrt(ss / ((double)N * (double)(N - 1))) : 0.0;

    // contraction path
    int prec = s->precision;
    if (!dense) {
        if (prec != SBQA_PREC_AUTO && prec != SBQA_PREC_FP32)
            return fail(SBQA_EINVAL, "CSR couplings support only fp32 precision");
        facts->path = PATH_CSR;
    } else {
        if (prec == SBQA_PREC_AUTO)
            prec = s->fmode == SBQA_F_BALLISTIC ? SBQA_PREC_FP32
                   : ternary                    ? SBQA_PREC_FP4
                   : facts->int8                ? SBQA_PREC_INT8
                                                : SBQA_PREC_FP32;
        if (prec == SBQA_PREC_FP8 || prec == SBQA_PREC_FP4) {
            const char *nm = prec == SBQA_PREC_FP8 ? "FP8" : "FP4";
            if (s->fmode == SBQA_F_BALLISTIC) return fail(SBQA_EINVAL, "%s precision needs ternary or sign f (ballistic operands are not exact)", nm);
            if (!ternary) return fail(SBQA_EINVAL, "%s precision needs J in {-1,0,+1}", nm);
        }
        if (prec == SBQA_PREC_INT8) {
            if (s->fmode == SBQA_F_BALLISTIC) return fail(SBQA_EINVAL, "INT8 precision needs ternary or sign f (ballistic operands are not integers)");
            if (!facts->int8) return fail(SBQA_EINVAL, "INT8 precision needs integer J with |J| <= 127");
        }
        const bool pack = facts->pm1 && s->j_packing == SBQA_JPACK_AUTO;
        facts->path = prec == SBQA_PREC_FP8      ? (pack ? PATH_FP8PK : PATH_FP8)
                      : prec == SBQA_PREC_FP4    ? (pack ? PATH_FP4PK : PATH_FP4)
                      : prec == SBQA_PREC_INT8   ? PATH_I8
                      : prec == SBQA_PREC_BF16X3 ? PATH_BF16X3
                                                 : PATH_F32;
    }
    return SBQA_OK;
}

void pack_sign_bits(const double *J, int32_t N, std::vector<uint32_t> *bits) {
    const int64_t words = (N + 31) / 32;
    bits->assign((size_t)(N * words), 0u);
    auto rows = [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t j = 0; j < N; ++j)
                if (J[i * N + j] < 0.0) (*bits)[(size_t)(i * words + j / 32)] |= 1u << (j % 32);
    };
    const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nt <= 1 || N < 512) {
        rows(0, N);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t per = (N + nt - 1) / nt;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back(rows, std::min<int64_t>(N, t * per), std::min<int64_t>(N, (t + 1) * per));
    for (std::thread &t : pool) t.join();
}

// Geometry and byte count of a context (also used by the server's admission).
void plan_layout(int32_t N, int32_t R, int32_t runs, const InstanceFacts &f, Layout *L) {
    const int64_t C = (int64_t)R * runs;
    L->C = (int)C;
    L->Cp = (int)round_up(C, GEMM_BM);
    // the operand is sized for the widest tile the autotuner may pick
    L->mbw = 4;
    L->Cg = (int)round_up(C, 64 * L->mbw);
    L->Np = (int)round_up(N, f.path == PATH_CSR ? GEMM_BN : dense_pad(f.path));
    L->Cs = (int)round_up(C, 4);
    L->esplits = 1;
    int64_t b = 0;
    if (f.path == PATH_CSR) {
        b += 2 * (int64_t)N * L->Cs * 4 + (int64_t)N * L->Cs * 4;        // x ping-pong, y
        b += 2 * (int64_t)N * L->Cs;                                      // int8 operand ping-pong
        b += (int64_t)(N + 1) * 4 + f.nnz * (4 + 4 + 8);                 // CSR
        b += (int64_t)N * 12;                                             // h32, h64
        // energy row blocks: at least one per reduction slot (ENERGY_SLOTS),
        // about 2048 blocks over the column chunks, >= 4 rows each
        const int64_t ncb = (C + 255) / 256;
        L->csr_nrb = (int)std::max<int64_t>(
            1, std::min<int64_t>((N + 3) / 4, std::max<int64_t>(ENERGY_SLOTS, (2048 + ncb - 1) / ncb)));
        // large instances: shorter row blocks (the first stage walks a
        // block's rows one after another, a chain of dependent loads per row),
        // at least 32 rows each, the partials within 64 MiB
        if (N > 65536)
            L->csr_nrb = (int)std::max<int64_t>(
                L->csr_nrb, std::min<int64_t>((N + 31) / 32, ((int64_t)64 << 20) / ((int64_t)C * 24)));
        b += (int64_t)L->csr_nrb * C * 24;
        if (f.n3) b += (int64_t)(N + 1) * 4 + 3 * f.n3 * (8 + 4 + 8);    // three-body lists
        b += (int64_t)N * L->Cs * 4;                                      // phi (fields hook)
    } else {
        const int planes = f.path == PATH_BF16X3 ? 2 : 1;
        L->nkc = dense_nkc(f.path, L->Np);
        const int64_t tiles = (int64_t)(L->Np / GEMM_BN) * (L->Cp / GEMM_BM);
        const int64_t nke = (int64_t)L->Np * 8 / GEMM_KB;
        int es = 1;
        while (tiles * es < 512 && es < 8 && nke % (2 * es) == 0 && nke / (2 * es) >= 4) es *= 2;
        L->esplits = es;
        b += 3 * C * (int64_t)L->Np * 4;                                  // x ping-pong, y
        b += 2 * dense_plane_bytes(f.path, L->Cg, L->Np) * planes;        // operand ping-pong
        b += dense_j_bytes(f.path, L->Np) * planes;                       // J
        if (f.jbits) b += (int64_t)N * ((N + 31) / 32) * 4;               // sign bits the J copy is built from
        else b += (int64_t)L->Np * L->Np * 8;                             // J fp64 (energies, source of J)
        b += (int64_t)L->Np * 12;                                         // h
        if (!path_energy_mfma(f.path)) b += (int64_t)L->Cp * L->Np * 8 * (1 + es);   // fp64 readout + energy partials
        L->csr_nrb = 0;
    }
    b += (int64_t)runs * (int64_t)0;  // schedule tables counted by the caller (steps known there)
    b += C * 8 + (int64_t)runs * (16 + N);                                // E, best
    L->bytes = (size_t)b;
}

void set_tile(Layout *L, int mbw) {
    L->mbw = mbw;
    L->Cg = (int)round_up(L->C, 64 * mbw);
}

// ------------------------------------------------------------ tile autotuner
// Dense workgroup tile: 64 * mbw replica columns (mbw m-blocks per wave).
// Candidates that pad C by at most 2x are timed once per (device, path, C, Np
// rounded up to a power of two), on scratch buffers of the instance's shape
// (the MFMA step's time does not depend on the values); the fastest is kept.
// Every tile sums each field in the same K order, so the choice never changes
// results. Choices persist across processes in a tile file (below), so a new
// process (a server restart) does not time them again.

// The device a choice was timed on: architecture and compute-unit count.
static std::string tile_device_tag() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "";
    static std::mutex mu;
    static std::map<int, std::string> tags;
    std::lock_guard<std::mutex> lk(mu);
    auto it = tags.find(dev);
    if (it != tags.end()) return it->second;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "";
    std::string arch(p.gcnArchName);
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    return tags[dev] = arch + " " + std::to_string(p.multiProcessorCount);
}

// The tile file: SBQA_TUNE_CACHE names it ("" or "off": choices stay in the
// process), else $XDG_CACHE_HOME/sbqa/dense_tiles.txt, else
// $HOME/.cache/sbqa/dense_tiles.txt. One line per choice,
//   sbqa-tile-v1 <arch> <CUs> <path> <C> <padded N> <mbw>
// appended with one write; unreadable files and malformed lines are ignored
// (a choice is used only when it is one of the key's candidates).
static std::string tile_file(bool make_dir) {
    const char *env = std::getenv("SBQA_TUNE_CACHE");
    if (env) return (std::strcmp(env, "off") == 0) ? std::string() : std::string(env);
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) dir = std::string(x) + "/sbqa";
    else if (const char *h = std::getenv("HOME"); h && *h) dir = std::string(h) + "/.cache/sbqa";
    else return std::string();
    if (make_dir) {
        const size_t cut = dir.rfind('/');
        if (cut != std::string::npos && cut > 0) (void)::mkdir(dir.substr(0, cut).c_str(), 0755);
        (void)::mkdir(dir.c_str(), 0755);
    }
    return dir + "/dense_tiles.txt";
}

static void load_tile_file(const std::string &dev, std::map<std::tuple<std::string, int, int, int>, int> *cache) {
    const std::string f = tile_file(false);
    if (f.empty()) return;
    FILE *fp = std::fopen(f.c_str(), "r");
    if (!fp) return;
    char line[512];
    while (std::fgets(line, sizeof line, fp)) {
        char tag[32], arch[256];
        int cus = 0, path = 0, C = 0, npb = 0, mbw = 0;
        if (std::sscanf(line, "%31s %255s %d %d %d %d %d", tag, arch, &cus, &path, &C, &npb, &mbw) != 7) continue;
        if (std::strcmp(tag, "sbqa-tile-v1") != 0 || std::string(arch) + " " + std::to_string(cus) != dev) continue;
        if (mbw == 1 || mbw == 2 || mbw == 4) (*cache)[std::make_tuple(dev, path, C, npb)] = mbw;
    }
    std::fclose(fp);
}

static void append_tile_file(const std::string &dev, int path, int C, int npb, int mbw) {
    const std::string f = tile_file(true);
    if (f.empty()) return;
    char line[512];
    const int n = std::snprintf(line, sizeof line, "sbqa-tile-v1 %s %d %d %d %d\n", dev.c_str(), path, C, npb, mbw);
    if (n <= 0 || n >= (int)sizeof line) return;
    const int fd = ::open(f.c_str(), O_WRONLY | O_APPEND | O_CREAT, 0644);
    if (fd < 0) return;
    (void)!::write(fd, line, (size_t)n);   // one append: whole lines, also from concurrent processes
    ::close(fd);
}

static int tune_dense_mbw(Path path, int C, int Np, hipStream_t st) {
    static std::mutex mu;
    static std::map<std::tuple<std::string, int, int, int>, int> cache;
    static std::set<std::string> loaded;
    int npb = 128;
    while (npb < Np) npb *= 2;
    const int fallback = dense_mbw(C);
    std::vector<int> cand;
    for (int m : {1, 2, 4})
        if (m == fallback || round_up(C, 64 * m) <= 2 * round_up(C, 64)) cand.push_back(m);
    const std::string dev = tile_device_tag();
    const auto key = std::make_tuple(dev, (int)path, C, npb);
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!dev.empty() && !loaded.count(dev)) {
            load_tile_file(dev, &cache);
            loaded.insert(dev);
        }
        auto it = cache.find(key);
        if (it != cache.end() && std::find(cand.begin(), cand.end(), it->second) != cand.end()) return it->second;
    }
    int best = fallback;
    bool timed = false;
    if (cand.size() > 1) {
        const int planes = path == PATH_BF16X3 ? 2 : 1;
        const int Cgm = (int)round_up(C, 256), nkc = dense_nkc(path, Np);
        std::vector<void *> bufs;
        auto grab = [&](size_t bytes) -> void * {
            void *p = nullptr;
            if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
            bufs.push_back(p);
            (void)hipMemsetAsync(p, 0, std::max<size_t>(bytes, 256), st);
            return p;
        };
        const size_t jb = (size_t)dense_j_bytes(path, Np), gb = (size_t)dense_plane_bytes(path, Cgm, Np),
                     sb = (size_t)C * Np * 4;
        DenseStepArgs a{};
        a.N = Np;
        a.Np = Np;
        a.R = 1;
        a.C = C;
        a.nkc = nkc;
        a.J = (const uint8_t *)grab(jb);
        a.J_lo = planes == 2 ? (const uint8_t *)grab(jb) : nullptr;
        a.g = (const uint8_t *)grab(gb);
        a.g_lo = planes == 2 ? (const uint8_t *)grab(gb) : nullptr;
        a.g_next = (uint8_t *)grab(gb);
        a.g_next_lo = planes == 2 ? (uint8_t *)grab(gb) : nullptr;
        a.h = (const float *)grab((size_t)Np * 4);
        a.x_in = (const float *)grab(sb);
        a.x_out = (float *)grab(sb);
        a.y = (float *)grab(sb);
        a.jp = (const float *)grab((size_t)C * 4);
        a.jp_stride = 1;
        a.fmode = 0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool ok = a.J && a.g && a.g_next && a.h && a.x_in && a.x_out && a.y && a.jp && (planes == 1 || (a.J_lo && a.g_lo && a.g_next_lo)) &&
                  hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
        float best_ms = 0.0f;
        for (int m : cand) {
            if (!ok) break;
            const int Cg = (int)round_up(C, 64 * m);
            ok = launch_dense_step(path, EPI_UPDATE, m, Cg, a, st) == hipSuccess;   // warm-up
            ok = ok && hipEventRecord(e0, st) == hipSuccess;
            for (int r = 0; r < 3 && ok; ++r) ok = launch_dense_step(path, EPI_UPDATE, m, Cg, a, st) == hipSuccess;
            ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (ok && (m == cand.front() || ms < best_ms)) {
                best_ms = ms;
                best = m;
            }
        }
        (void)hipStreamSynchronize(st);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (void *p : bufs) (void)hipFree(p);
        if (!ok) best = fallback;
        timed = ok;
        (void)hipGetLastError();
    }
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = best;
    if (timed && !dev.empty()) append_tile_file(dev, (int)path, C, npb, best);
    return best;
}

size_t instance_bytes(int32_t N, int32_t R, int32_t runs, const InstanceFacts &f, uint32_t steps) {
    Layout L;
    plan_layout(N, R, runs, f, &L);
    return L.bytes + ((size_t)runs + 2) * steps * 4 + 4;   // + J_perp table, per-step a_n and Delta_n tables
}

// ----------------------------------------------------------------- schedules
void build_schedule_host(const sbqa_schedule *s, int32_t runs, std::vector<double> &beta, std::vector<double> &alpha,
                         std::vector<float> &jp) {
    const uint32_t S = s->steps;
    beta.assign(runs, 0.0);
    alpha.assign(runs, 0.0);
    uint64_t st = s->seed ^ 0xA5A5F00DBAADC0DEull;
    for (int r = 0; r < runs; ++r) {
        const double u1 = unit_double(st), u2 = unit_double(st);
        beta[r] = s->beta ? s->beta[r] : s->beta_lo + (s->beta_hi - s->beta_lo) * u1;
        alpha[r] = s->alpha ? s->alpha[r] : s->alpha_lo + (s->alpha_hi - s->alpha_lo) * u2;
    }
    jp.assign((size_t)runs * S, 0.0f);
    for (int r = 0; r < runs; ++r)
        for (uint32_t n = 0; n < S; ++n) {
            const double sn = (double)n / (double)S;   // t/T at the start of step n
            double v;
            if (s->jp_kind == SBQA_JP_LINEAR) v = s->jp_start + (s->jp_end - s->jp_start) * sn;
            else if (s->jp_kind == SBQA_JP_PAPER) {
                const double gx = s->gamma0_over_R * (std::pow(1.0 - sn, alpha[r]) + 1e-5);  // Eq. 5
                v = -std::log(std::tanh(beta[r] * gx)) / (2.0 * beta[r]);
            } else v = s->jp_table[(size_t)r * S + n];
            jp[(size_t)r * S + n] = (float)v;
        }
}

StepCoef step_coef(const sbqa_schedule *s, double c0, int R, uint32_t n) {
    const double S = (double)s->steps;
    StepCoef k;
    k.kA = (float)((s->a0 - (double)n / S) / (double)R);
    k.kB = (float)(c0 / (double)R);
    k.dt = (float)s->dt;
    k.kD = (float)(s->dt * s->a0 / (double)R);
    k.delta_next = (float)((s->delta_max * (double)(n + 1)) / S);
    return k;
}

float delta_at(const sbqa_schedule *s, uint32_t n) {
    return (float)((s->delta_max * (double)n) / (double)s->steps);
}

}  // namespace sbqa

using namespace sbqa;

// =========================================================================== //
//                                 context                                     //
// =========================================================================== //

sbqa_ctx::~sbqa_ctx() {
    for (void *p : allocs) (void)hipFree(p);
    if (rhost) (void)hipHostFree(rhost);
}

template <class T>
static hipError_t dalloc(sbqa_ctx *c, T **p, size_t n) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(n * sizeof(T), 256);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return e;
    c->allocs.push_back(q);
    c->bytes += bytes;
    e = hipMemsetAsync(q, 0, bytes, c->stream);
    *p = static_cast<T *>(q);
    return e;
}

static sbqa_status check_device(int *dev) {
    HIP_TRY(hipGetDevice(dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, *dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SBQA_EDEVICE, "device %d is %s; this library is built for gfx950 (MI355X) only", *dev,
                    prop.gcnArchName);
    return SBQA_OK;
}

namespace sbqa {

// Elements of one state buffer (x or y) including padding.
static size_t state_elems(const sbqa_ctx *c) {
    if (c->order == ORDER_REPLICA_MAJOR) return (size_t)c->L.C * c->ld;
    if (c->order == ORDER_COLBLOCK8) return (size_t)c->L.C * c->ld;
    return (size_t)c->N * c->ld;
}

// Build operand f(X) of the current step from the current state.
sbqa_status rebuild_operand(sbqa_ctx *c) {
    const float d = delta_at(&c->s, c->step);
    if (c->facts.path == PATH_CSR) {
        // elementwise over the whole buffer: column-block order has C == Cs
        // and zero padded rows, whose operand is 0
        // (the resident loop builds its operand from x at each launch)
        if (c->s.fmode != SBQA_F_BALLISTIC && !c->resident)
            HIP_TRY(launch_csr_operand(c->s.fmode, c->N, c->L.Cs, c->L.C, c->x[c->cur], (int8_t *)c->g[c->cur], d,
                                       c->stream));
    } else {
        HIP_TRY(launch_dense_operand(c->facts.path, c->s.fmode, c->N, c->L.Np, c->L.C, c->L.nkc, c->L.mbw, c->x[c->cur],
                                     c->g[c->cur], c->g_lo[c->cur], d, c->stream));
    }
    return SBQA_OK;
}

sbqa_status ctx_upload(sbqa_ctx *c, const sbqa_coupling *J, const double *h, const uint32_t *jbits) {
    const int N = c->N, Np = c->L.Np, Cs = c->L.Cs, C = c->L.C, Cp = c->L.Cp;
    const Path path = c->facts.path;
    const int runs = c->runs;
    const uint32_t S = c->s.steps;
    HIP_TRY(dalloc(c, &c->jp, (size_t)runs * S));
    HIP_TRY(hipMemcpyAsync(c->jp, c->jp_host.data(), sizeof(float) * runs * S, hipMemcpyHostToDevice, c->stream));
    {
        // per-step pump and threshold tables (a_n term and Delta_n of Eq. 8),
        // read on the device by the resident loops and the grouped steps
        std::vector<float> ca(S), dtab((size_t)S + 1);
        for (uint32_t n = 0; n < S; ++n) ca[n] = step_coef(&c->s, c->c0, c->R, n).kA;
        for (uint32_t n = 0; n <= S; ++n) dtab[n] = delta_at(&c->s, n);
        HIP_TRY(dalloc(c, &c->coefA, ca.size()));
        HIP_TRY(dalloc(c, &c->delta_tab, dtab.size()));
        HIP_TRY(hipMemcpyAsync(c->coefA, ca.data(), sizeof(float) * ca.size(), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->delta_tab, dtab.data(), sizeof(float) * dtab.size(), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));   // host staging buffers die here
    }
    HIP_TRY(dalloc(c, &c->E, (size_t)std::max(C, Cp)));
    HIP_TRY(dalloc(c, &c->bestStep, (size_t)runs));
    if (N > BEST_SPLIT_N) HIP_TRY(dalloc(c, &c->bsel, (size_t)runs));
    c->rbytes = (size_t)8 * runs + 8 + (size_t)runs * N;
    HIP_TRY(dalloc(c, &c->rdev, c->rbytes));
    HIP_TRY(hipHostMalloc((void **)&c->rhost, c->rbytes, hipHostMallocCoherent));
    std::memset(c->rhost, 0, c->rbytes);
    {
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, c->rhost, 0) == hipSuccess) c->rhost_dev = static_cast<uint8_t *>(dp);
        else (void)hipGetLastError();   // keep the copy engine path
    }
    c->bestE = reinterpret_cast<double *>(c->rdev);
    c->err = reinterpret_cast<int *>(c->rdev + (size_t)8 * runs);
    c->bestSpins = reinterpret_cast<int8_t *>(c->rdev + (size_t)8 * runs + 8);

    const int hrows = std::max(Np, c->resident ? c->res_rows : 0);
    std::vector<float> h32((size_t)hrows, 0.0f);
    std::vector<double> h64((size_t)N, 0.0);
    if (h)
        for (int i = 0; i < N; ++i) {
            h32[i] = (float)h[i];
            h64[i] = h[i];
        }
    HIP_TRY(dalloc(c, &c->h32, (size_t)hrows));
    HIP_TRY(dalloc(c, &c->h64, (size_t)N));
    HIP_TRY(hipMemcpyAsync(c->h32, h32.data(), sizeof(float) * hrows, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h64, h64.data(), sizeof(double) * N, hipMemcpyHostToDevice, c->stream));
    c->has_h = h != nullptr;

    if (path == PATH_CSR) {
        const int64_t nnz = J->nnz;
        const int rows = c->resident ? c->res_rows : N;   // resident rows are padded with zero rows
        HIP_TRY(dalloc(c, &c->x[0], (size_t)rows * Cs));
        HIP_TRY(dalloc(c, &c->y, (size_t)rows * Cs));
        // the resident loop steps x in place and builds its operand on chip:
        // the second state half, the operand buffers and the fields buffer
        // are only the fields hook's scratch there, allocated at its first call
        if (!c->resident) {
            HIP_TRY(dalloc(c, &c->x[1], (size_t)rows * Cs));
            int8_t *g0, *g1;
            HIP_TRY(dalloc(c, &g0, (size_t)rows * Cs));
            HIP_TRY(dalloc(c, &g1, (size_t)rows * Cs));
            c->g[0] = g0;
            c->g[1] = g1;
        }
        HIP_TRY(dalloc(c, &c->rp, (size_t)N + 1));
        // +8: the CSR step reads neighbour indices in batches of up to 8
        HIP_TRY(dalloc(c, &c->col, (size_t)nnz + 8));
        HIP_TRY(dalloc(c, &c->val, (size_t)nnz + 8));
        HIP_TRY(dalloc(c, &c->val64, (size_t)nnz));
        // row-block partials of the spin-major energies (the column-block
        // readout of a resident context reduces on chip)
        if (c->order != ORDER_COLBLOCK8 || J->n3 > 0)
            HIP_TRY(dalloc(c, &c->csr_partial, (size_t)c->L.csr_nrb * C * 3));
        if (J->n3 > 0) {
            // three-body terms listed per member spin, triples in the given
            // order; +4 entries: the step reads them in batches of up to 4
            std::vector<int32_t> tp((size_t)N + 1, 0);
            for (int64_t t = 0; t < J->n3; ++t)
                for (int e = 0; e < 3; ++e) ++tp[(size_t)J->tri[3 * t + e] + 1];
            for (int32_t i = 0; i < N; ++i) tp[(size_t)i + 1] += tp[(size_t)i];
            const int64_t ne = 3 * J->n3;
            std::vector<int32_t> ab((size_t)2 * (ne + 4), 0), fill(tp.begin(), tp.end() - 1);
            std::vector<float> k32((size_t)ne + 4, 0.0f);
            std::vector<double> k64((size_t)ne, 0.0);
            for (int64_t t = 0; t < J->n3; ++t)
                for (int e = 0; e < 3; ++e) {
                    const int32_t *v = J->tri + 3 * t;
                    const int64_t q = fill[(size_t)v[e]]++;
                    ab[(size_t)2 * q] = v[(e + 1) % 3];
                    ab[(size_t)2 * q + 1] = v[(e + 2) % 3];
                    k32[(size_t)q] = (float)J->K[t];
                    k64[(size_t)q] = J->K[t];
                }
            HIP_TRY(dalloc(c, &c->t3ptr, tp.size()));
            HIP_TRY(dalloc(c, &c->t3ab, ab.size()));
            HIP_TRY(dalloc(c, &c->t3k, k32.size()));
            HIP_TRY(dalloc(c, &c->t3k64, k64.size()));
            HIP_TRY(hipMemcpyAsync(c->t3ptr, tp.data(), sizeof(int32_t) * tp.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipMemcpyAsync(c->t3ab, ab.data(), sizeof(int32_t) * ab.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipMemcpyAsync(c->t3k, k32.data(), sizeof(float) * k32.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipMemcpyAsync(c->t3k64, k64.data(), sizeof(double) * k64.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));   // host staging buffers die here
        }
        if (!c->resident) HIP_TRY(dalloc(c, &c->phi, (size_t)N * Cs));
        std::vector<float> v32((size_t)nnz);
        for (int64_t p = 0; p < nnz; ++p) v32[p] = (float)J->val[p];
        HIP_TRY(hipMemcpyAsync(c->rp, J->row_ptr, sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->col, J->col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->val, v32.data(), sizeof(float) * nnz, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->val64, J->val, sizeof(double) * nnz, hipMemcpyHostToDevice, c->stream));
        std::vector<int32_t> cp, rc;
        std::vector<float> vp;
        std::vector<double> rv, rhv;
        if (c->resident) {
            // padded neighbour lists (CSR order, then index 0 with weight 0),
            // ring exchange buffers
            const int D = c->res_D, NR = c->res_rows;
            cp.assign((size_t)NR * D, 0);
            vp.assign((size_t)D * NR, 0.0f);
            for (int i = 0; i < N; ++i)
                for (int q = 0; q < J->row_ptr[i + 1] - J->row_ptr[i]; ++q) {
                    cp[(size_t)i * D + q] = J->col[J->row_ptr[i] + q];
                    vp[(size_t)q * NR + i] = (float)J->val[J->row_ptr[i] + q];
                }
            // the readout energies' copy, grouped by the energy row blocks:
            // [row in block][neighbour][row block]
            const int nrb = c->L.csr_nrb, rpb = (N + nrb - 1) / nrb, RS = energy_colblock_rows(rpb);
            rc.assign((size_t)nrb * RS * D, 0);
            rv.assign((size_t)nrb * RS * D, 0.0);
            rhv.assign((size_t)nrb * RS, 0.0);
            for (int i = 0; i < N; ++i) {
                const size_t rb = (size_t)(i / rpb), r = (size_t)(i % rpb);
                for (int q = 0; q < J->row_ptr[i + 1] - J->row_ptr[i]; ++q) {
                    rc[(r * D + q) * nrb + rb] = J->col[J->row_ptr[i] + q];
                    rv[(r * D + q) * nrb + rb] = J->val[J->row_ptr[i] + q];
                }
                if (h) rhv[r * nrb + rb] = h[i];
            }
            HIP_TRY(dalloc(c, &c->colpad, cp.size()));
            HIP_TRY(dalloc(c, &c->valpad, vp.size()));
            HIP_TRY(dalloc(c, &c->rcol, rc.size()));
            HIP_TRY(dalloc(c, &c->rval, rv.size()));
            HIP_TRY(dalloc(c, &c->rh, rhv.size()));
            HIP_TRY(hipMemcpyAsync(c->rcol, rc.data(), sizeof(int32_t) * rc.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipMemcpyAsync(c->rval, rv.data(), sizeof(double) * rv.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipMemcpyAsync(c->rh, rhv.data(), sizeof(double) * rhv.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(dalloc(c, &c->xpub, (size_t)2 * c->res_nwg * 2 * NR));
            HIP_TRY(dalloc(c, &c->flags, (size_t)c->res_nwg));
            HIP_TRY(dalloc(c, &c->epoch_cnt, (size_t)c->res_nwg));
            HIP_TRY(dalloc(c, &c->sbits, (size_t)c->res_nwg * NR));
            HIP_TRY(dalloc(c, &c->rd_cnt, (size_t)runs));
            HIP_TRY(hipMemcpyAsync(c->colpad, cp.data(), sizeof(int32_t) * cp.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipMemcpyAsync(c->valpad, vp.data(), sizeof(float) * vp.size(), hipMemcpyHostToDevice, c->stream));
        }
        HIP_TRY(hipStreamSynchronize(c->stream));   // host staging buffers die here
        return SBQA_OK;
    }

    const int nkc = c->L.nkc, Cg = c->L.Cg;
    const size_t gbytes = (size_t)dense_plane_bytes(path, Cg, Np);
    HIP_TRY(dalloc(c, &c->x[0], (size_t)C * Np));
    HIP_TRY(dalloc(c, &c->x[1], (size_t)C * Np));
    HIP_TRY(dalloc(c, &c->y, (size_t)C * Np));
    for (int q = 0; q < 2; ++q) {
        uint8_t *gb, *glo = nullptr;
        HIP_TRY(dalloc(c, &gb, gbytes));
        if (path == PATH_BF16X3) HIP_TRY(dalloc(c, &glo, gbytes));
        c->g[q] = gb;
        c->g_lo[q] = glo;
    }
    if (!path_energy_mfma(path)) {   // float64 readout spins and energy GEMM partials
        HIP_TRY(dalloc(c, &c->S64, (size_t)Cp * Np));
        HIP_TRY(dalloc(c, &c->phis64, (size_t)c->L.esplits * Cp * Np));
    }
    if (c->resident) {
        // small dense loop: J float32 [N][N]
        std::vector<float> jsm((size_t)N * N);
        for (size_t q = 0; q < jsm.size(); ++q) jsm[q] = (float)J->dense[q];
        HIP_TRY(dalloc(c, &c->Jsm, jsm.size()));
        HIP_TRY(hipMemcpyAsync(c->Jsm, jsm.data(), sizeof(float) * jsm.size(), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));   // host staging buffers die here
    }

    if (c->facts.jbits) {
        // +-1 J as sign bits: the bit-packed contraction copy is built from
        // them; no float64 copy (the readout energies run on MFMA)
        if (!jbits || !path_packed(path)) return fail(SBQA_EINVAL, "sign bits need a bit-packed +-1 path");
        uint8_t *jd;
        uint32_t *sb;
        const size_t words = (size_t)(N + 31) / 32;
        HIP_TRY(dalloc(c, &jd, (size_t)dense_j_bytes(path, Np)));
        HIP_TRY(dalloc(c, &sb, (size_t)N * words));
        c->Jd = jd;
        HIP_TRY(hipMemcpyAsync(sb, jbits, sizeof(uint32_t) * N * words, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(launch_convert_j_bits(path, sb, N, Np, nkc, jd, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));   // the caller may free the bits on return
        return SBQA_OK;
    }
    // J in the contraction precision (fragment-tiled) and in float64
    // (row-major, energies), zero padded.
    const double *A = J->dense;
    uint8_t *jd, *jlo = nullptr;
    double *j64;
    HIP_TRY(dalloc(c, &jd, (size_t)dense_j_bytes(path, Np)));
    if (path == PATH_BF16X3) HIP_TRY(dalloc(c, &jlo, (size_t)dense_j_bytes(path, Np)));
    HIP_TRY(dalloc(c, &j64, (size_t)Np * Np));
    c->Jd = jd;
    c->Jd_lo = jlo;
    c->J64 = j64;
    // float64 J into the zero-padded row-major copy (energies), then the
    // contraction copy is derived from it on the device. The host array goes
    // up in one contiguous copy (a pitched copy from pageable memory is split
    // into one transfer per row); when rows need padding it lands in a
    // temporary buffer first and is spread into the padded rows on the GPU.
    if (N == Np) {
        HIP_TRY(hipMemcpyAsync(j64, A, sizeof(double) * N * N, hipMemcpyHostToDevice, c->stream));
    } else {
        double *tmp = nullptr;
        HIP_TRY(hipMalloc(&tmp, sizeof(double) * (size_t)N * N));
        struct Tmp { double *p; ~Tmp() { (void)hipFree(p); } } guard{tmp};
        HIP_TRY(hipMemcpyAsync(tmp, A, sizeof(double) * N * N, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(launch_pad_rows(tmp, N, Np, j64, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));   // tmp is freed at return
    }
    HIP_TRY(launch_convert_j(path, j64, Np, nkc, jd, jlo, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));   // the caller may free J on return
    return SBQA_OK;
}

// Arguments of the dense step kernel at step n from operand/state buffer `in`.
static DenseStepArgs dense_args(sbqa_ctx *c, uint32_t n, int in) {
    DenseStepArgs a{};
    a.N = c->N;
    a.Np = c->L.Np;
    a.R = c->R;
    a.C = c->L.C;
    a.nkc = c->L.nkc;
    a.reverse = (int)(n & 1u);
    a.J = static_cast<const uint8_t *>(c->Jd);
    a.J_lo = static_cast<const uint8_t *>(c->Jd_lo);
    a.g = static_cast<const uint8_t *>(c->g[in]);
    a.g_lo = static_cast<const uint8_t *>(c->g_lo[in]);
    a.g_next = static_cast<uint8_t *>(c->g[1 - in]);
    a.g_next_lo = static_cast<uint8_t *>(c->g_lo[1 - in]);
    a.h = c->h32;
    a.x_in = c->x[in];
    a.x_out = c->x[1 - in];
    a.y = c->y;
    a.phi = nullptr;
    a.jp = c->jp + (n < c->s.steps ? n : 0);
    a.jp_stride = c->s.steps;
    a.k = step_coef(&c->s, c->c0, c->R, n);
    a.fmode = c->s.fmode;
    return a;
}

// One step of Eqs. 6-7 on the device (asynchronous).
sbqa_status ctx_step_once(sbqa_ctx *c) {
    const uint32_t n = c->step;
    const StepCoef k = step_coef(&c->s, c->c0, c->R, n);
    const float *jp = c->jp + n;
    const int64_t jp_stride = c->s.steps;
    const int in = c->cur, out = 1 - c->cur;
    if (c->facts.path == PATH_CSR) {
        HIP_TRY(launch_csr_step(c->s.fmode, c->N, c->L.Cs, c->R, c->runs, c->rp, c->col, c->val, c->tri3(), c->h32, c->x[in],
                                c->x[out], c->y, (const int8_t *)c->g[in], (int8_t *)c->g[out], jp, jp_stride, k,
                                c->stream));
    } else {
        const DenseStepArgs a = dense_args(c, n, in);
        HIP_TRY(launch_dense_step(c->facts.path, EPI_UPDATE, c->L.mbw, c->L.Cg, a, c->stream));
    }
    c->cur = out;
    c->step = n + 1;
    return SBQA_OK;
}

// The sign bytes the resident loop wrote for the current state, or nullptr
// when the state has been replaced since.
static const uint8_t *colblock_signs(const sbqa_ctx *c) {
    return c->sbits_step == (int64_t)c->step ? c->sbits : nullptr;
}

// Energies of the readout of the current state into c->E[0..C).
sbqa_status ctx_state_energies(sbqa_ctx *c) {
    const bool sm = c->facts.path == PATH_CSR;
    const double *h64 = c->has_h ? c->h64 : nullptr;
    if (sm && c->order == ORDER_COLBLOCK8 && !c->facts.n3) {
        const int nrb = c->L.csr_nrb, rpb = (c->N + nrb - 1) / nrb;
        HIP_TRY(launch_csr_energy_colblock(c->N, c->ld, c->L.C, c->res_D, nrb, rpb, c->rcol, c->rval, c->rh,
                                           c->x[c->cur], colblock_signs(c), c->E, c->stream));
    } else if (sm) {
        HIP_TRY(launch_csr_energy_state(c->N, c->order, c->ld, c->L.C, c->rp, c->col, c->val64, c->tri3(), h64, c->x[c->cur],
                                        c->csr_partial, c->L.csr_nrb, c->E, c->stream));
    } else if (c->facts.path == PATH_FP8 || c->facts.path == PATH_FP8PK || c->facts.path == PATH_I8 ||
               path_fp4(c->facts.path)) {
        // integer J: J s on MFMA is exact, so the energies equal the float64
        // ones bit for bit; the free halves of the ping-pong buffers (written
        // in full by the next step before they are read) hold the readout
        // operand and its fields
        const int in = c->cur, sc = 1 - c->cur;
        HIP_TRY(launch_readout_operand(c->facts.path, c->N, c->L.Np, c->L.C, c->L.nkc, c->L.mbw, c->x[in], c->g[sc],
                                       c->stream));
        DenseStepArgs a = dense_args(c, c->step, in);
        a.g = static_cast<const uint8_t *>(c->g[sc]);
        a.phi = c->x[sc];
        HIP_TRY(launch_dense_step(c->facts.path, EPI_FIELDS, c->L.mbw, c->L.Cg, a, c->stream));
        HIP_TRY(launch_energy_fields(c->N, c->L.Np, c->L.C, c->x[in], c->x[sc], h64, c->E, c->stream));
    } else {
        HIP_TRY(launch_readout_f64(c->N, c->L.Np, c->L.C, c->L.Np, false, c->x[c->cur], c->S64, c->stream));
        HIP_TRY(launch_gemm_f64(c->S64, c->J64, c->phis64, c->L.Np, c->L.Cp, c->L.esplits, c->stream));
        HIP_TRY(launch_energy_reduce(c->N, c->L.Np, c->L.C, c->L.Cp, c->L.esplits, c->phis64, c->S64, h64, c->E, c->stream));
    }
    return SBQA_OK;
}

EnergyGemm energy_gemm(const sbqa_ctx *c, int count) {
    EnergyGemm g;
    const int Np = c->L.Np;
    g.cp = (int)round_up(count, GEMM_BM);
    const int64_t tiles = (int64_t)(Np / GEMM_BN) * (g.cp / GEMM_BM);
    const int64_t nke = (int64_t)Np * 8 / GEMM_KB;
    g.es = 1;
    while (tiles * g.es < 512 && g.es < 8 && nke % (2 * g.es) == 0 && nke / (2 * g.es) >= 4) g.es *= 2;
    return g;
}

sbqa_status ctx_energies_dev(sbqa_ctx *c, const int8_t *ds, int32_t count, double *E, double *S, double *P) {
    const int N = c->N;
    if (c->facts.path != PATH_CSR && !c->J64)
        return fail(SBQA_EINVAL, "this context keeps no float64 copy of J (built from sign bits)");
    const double *h64 = c->has_h ? c->h64 : nullptr;
    if (c->facts.path == PATH_CSR) {
        HIP_TRY(launch_csr_energy_spins(N, count, c->rp, c->col, c->val64, c->tri3(), h64, ds, E, c->stream));
    } else {
        const EnergyGemm g = energy_gemm(c, count);
        HIP_TRY(launch_spins_to_f64(N, c->L.Np, count, ds, S, c->stream));
        HIP_TRY(launch_gemm_f64(S, c->J64, P, c->L.Np, g.cp, g.es, c->stream));
        HIP_TRY(launch_energy_reduce(N, c->L.Np, count, g.cp, g.es, P, S, h64, E, c->stream));
    }
    return SBQA_OK;
}

sbqa_status ctx_evaluate(sbqa_ctx *c, bool reset) {
    sbqa_status st = ctx_state_energies(c);
    if (st != SBQA_OK) return st;
    HIP_TRY(launch_best_update(c->N, c->R, c->runs, c->order, c->ld, c->x[c->cur], c->E, c->bestE, c->bestStep,
                               c->bestSpins, (int64_t)c->step, reset, c->bsel, c->stream));
    c->last_eval_step = c->step;
    return SBQA_OK;
}

sbqa_status ctx_reset_best(sbqa_ctx *c) {
    std::vector<double> inf((size_t)c->runs, INFINITY);
    HIP_TRY(hipMemcpyAsync(c->bestE, inf.data(), sizeof(double) * c->runs, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->last_eval_step = -1;
    return SBQA_OK;
}

// Whether the register-resident CSR loop fits this instance on this device.
static bool resident_plan(sbqa_ctx *c, const sbqa_coupling *J, std::string *why) {
    if (c->s.fmode == SBQA_F_BALLISTIC) { *why = "ballistic f needs a float32 operand"; return false; }
    if (c->facts.n3) { *why = "three-body terms run on the streaming kernel"; return false; }
    if (c->R % resident_cols()) { *why = "R is not a multiple of 8"; return false; }
    const int rpt = resident_rpt(c->N);
    if (rpt < 0 || c->N > 65535) { *why = "N above 4096"; return false; }
    int maxdeg = 0;
    for (int i = 0; i < c->N; ++i) maxdeg = std::max(maxdeg, J->row_ptr[i + 1] - J->row_ptr[i]);
    const int D = resident_degree(maxdeg);
    if (D < 0) { *why = "degree above 16"; return false; }
    if (resident_rows(c->N) > 2048 && D > 6) { *why = "N above 2048 with degree above 6 exceeds the register budget"; return false; }
    const size_t lds = resident_lds_bytes(c->N, D);
    if (lds > 160 * 1024) { *why = "LDS demand above 160 KiB"; return false; }
    int bpc = 0, cus = 0;
    if (resident_max_blocks(D, c->N, &bpc) != hipSuccess) { *why = "occupancy query failed"; return false; }
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) { *why = "no CU count"; return false; }
    const int nwg = c->L.C / resident_cols();
    if (nwg > bpc * cus) { *why = "more column blocks than co-resident workgroups"; return false; }
    c->res_D = D;
    c->res_rows = resident_rows(c->N);
    c->res_nwg = nwg;
    return true;
}

// Whether the small dense resident loop fits this instance.
static bool small_plan(sbqa_ctx *c, std::string *why) {
    if (c->facts.path == PATH_BF16X3) { *why = "the small dense loop computes in float32 (every precision but BF16X3)"; return false; }
    if (c->N > SMALL_MAX_N) { *why = "N is above the small dense loop's limit"; return false; }
    if ((int64_t)c->R * c->N > SMALL_MAX_ELEMS) { *why = "R*N is above the small dense loop's limit"; return false; }
    if (small_lds_bytes(c->N, c->R) > 160 * 1024) { *why = "the run state does not fit in LDS"; return false; }
    return true;
}

// ---------------------------------------------------------------------------
// Internal relabelling of CSR spins for cache locality (sbqa_reorder).
// ---------------------------------------------------------------------------

// Undirected adjacency of the pairs and of the triples' members, as offsets
// and neighbour lists (duplicates allowed).
static void spin_adjacency(const sbqa_coupling *J, int32_t N, std::vector<int64_t> *aptr, std::vector<int32_t> *adj) {
    std::vector<int64_t> deg((size_t)N + 1, 0);
    for (int32_t i = 0; i < N; ++i) deg[(size_t)i + 1] += J->row_ptr[i + 1] - J->row_ptr[i];
    for (int64_t t = 0; t < J->n3; ++t)
        for (int e = 0; e < 3; ++e) deg[(size_t)J->tri[3 * t + e] + 1] += 2;
    for (int32_t i = 0; i < N; ++i) deg[(size_t)i + 1] += deg[(size_t)i];
    adj->assign((size_t)deg[(size_t)N], 0);
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int32_t i = 0; i < N; ++i)
        for (int32_t p = J->row_ptr[i]; p < J->row_ptr[i + 1]; ++p) (*adj)[(size_t)fill[(size_t)i]++] = J->col[p];
    for (int64_t t = 0; t < J->n3; ++t)
        for (int e = 0; e < 3; ++e) {
            const int32_t *v = J->tri + 3 * t;
            (*adj)[(size_t)fill[(size_t)v[e]]++] = v[(e + 1) % 3];
            (*adj)[(size_t)fill[(size_t)v[e]]++] = v[(e + 2) % 3];
        }
    *aptr = std::move(deg);
}

// Mean |label(i) - label(j)| over the adjacency (label = identity when pnew
// is empty).
static double mean_span(const std::vector<int64_t> &aptr, const std::vector<int32_t> &adj, int32_t N,
                        const std::vector<int32_t> &pnew) {
    if (adj.empty()) return 0.0;
    double sum = 0.0;
    for (int32_t i = 0; i < N; ++i)
        for (int64_t p = aptr[(size_t)i]; p < aptr[(size_t)i + 1]; ++p) {
            const int32_t j = adj[(size_t)p];
            sum += pnew.empty() ? std::fabs((double)i - j) : std::fabs((double)pnew[(size_t)i] - pnew[(size_t)j]);
        }
    return sum / (double)adj.size();
}

// Reverse Cuthill-McKee order: breadth-first through every connected
// component, each started at its lowest-degree unvisited spin, neighbours
// taken by increasing degree; the whole order reversed. pnew[i] = new label.
static void rcm_order(const std::vector<int64_t> &aptr, const std::vector<int32_t> &adj, int32_t N,
                      std::vector<int32_t> *pnew) {
    std::vector<int32_t> byDeg((size_t)N), order;
    order.reserve((size_t)N);
    for (int32_t i = 0; i < N; ++i) byDeg[(size_t)i] = i;
    auto deg = [&](int32_t i) { return aptr[(size_t)i + 1] - aptr[(size_t)i]; };
    std::stable_sort(byDeg.begin(), byDeg.end(), [&](int32_t a, int32_t b) { return deg(a) < deg(b); });
    std::vector<char> seen((size_t)N, 0);
    std::vector<int32_t> nb;
    for (int32_t start : byDeg) {
        if (seen[(size_t)start]) continue;
        seen[(size_t)start] = 1;
        size_t head = order.size();
        order.push_back(start);
        while (head < order.size()) {
            const int32_t u = order[head++];
            nb.clear();
            for (int64_t p = aptr[(size_t)u]; p < aptr[(size_t)u + 1]; ++p) {
                const int32_t v = adj[(size_t)p];
                if (!seen[(size_t)v]) { seen[(size_t)v] = 1; nb.push_back(v); }
            }
            std::stable_sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg(a) < deg(b); });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    pnew->assign((size_t)N, 0);
    for (int32_t k = 0; k < N; ++k) (*pnew)[(size_t)order[(size_t)(N - 1 - k)]] = k;
}

// Whether (and how) to relabel a CSR instance's spins (sbqa_reorder).
static void plan_reorder(const sbqa_coupling *J, int32_t N, int mode, std::vector<int32_t> *pnew) {
    pnew->clear();
    if (mode == SBQA_REORDER_OFF || (J->nnz == 0 && J->n3 == 0)) return;
    if (mode == SBQA_REORDER_AUTO && N < 16384) return;
    std::vector<int64_t> aptr;
    std::vector<int32_t> adj;
    spin_adjacency(J, N, &aptr, &adj);
    const double before = mean_span(aptr, adj, N, {});
    if (mode == SBQA_REORDER_AUTO && before <= (double)N / 64.0) return;
    std::vector<int32_t> p;
    rcm_order(aptr, adj, N, &p);
    if (mode == SBQA_REORDER_AUTO && mean_span(aptr, adj, N, p) * 4.0 > before) return;
    *pnew = std::move(p);
}

// The coupling with spins relabelled by pnew: row pnew[i] holds spin i's
// couplings in the given order (columns relabelled), triples keep their
// order with relabelled members; h permuted alike. The vectors own the data.
struct Relabelled {
    std::vector<int32_t> rp, col, tri;
    std::vector<double> val, h;
    sbqa_coupling J{};
};
static void relabel(const sbqa_coupling *J, const double *h, int32_t N, const std::vector<int32_t> &pnew,
                    Relabelled *r) {
    std::vector<int32_t> orig((size_t)N);
    for (int32_t i = 0; i < N; ++i) orig[(size_t)pnew[(size_t)i]] = i;
    r->rp.assign((size_t)N + 1, 0);
    for (int32_t k = 0; k < N; ++k) {
        const int32_t i = orig[(size_t)k];
        r->rp[(size_t)k + 1] = r->rp[(size_t)k] + (J->row_ptr[i + 1] - J->row_ptr[i]);
    }
    r->col.resize((size_t)J->nnz);
    r->val.resize((size_t)J->nnz);
    for (int32_t k = 0; k < N; ++k) {
        const int32_t i = orig[(size_t)k];
        int64_t q = r->rp[(size_t)k];
        for (int32_t p = J->row_ptr[i]; p < J->row_ptr[i + 1]; ++p, ++q) {
            r->col[(size_t)q] = pnew[(size_t)J->col[p]];
            r->val[(size_t)q] = J->val[p];
        }
    }
    r->tri.resize((size_t)3 * J->n3);
    for (int64_t q = 0; q < 3 * J->n3; ++q) r->tri[(size_t)q] = pnew[(size_t)J->tri[q]];
    if (h) {
        r->h.resize((size_t)N);
        for (int32_t i = 0; i < N; ++i) r->h[(size_t)pnew[(size_t)i]] = h[i];
    }
    r->J = *J;
    r->J.row_ptr = r->rp.data();
    r->J.col = r->col.data();
    r->J.val = r->val.data();
    r->J.tri = J->n3 ? r->tri.data() : nullptr;
}

// The stream of the contexts created without one: one non-blocking stream per
// device, created at the first such context and kept until the process ends
// (a stream per context cost a hardware queue's creation, 3.5 ms, for each of
// the first few contexts of a process). Their work is ordered on it;
// sbqa_set_stream gives a context a stream of the caller's.
static hipError_t library_stream(int device, hipStream_t *out) {
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(device);
    if (it != streams.end()) {
        *out = it->second;
        return hipSuccess;
    }
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    streams[device] = st;
    *out = st;
    return hipSuccess;
}

sbqa_status ctx_create(const sbqa_coupling *J, const double *h, int32_t N, int32_t R, int32_t runs,
                       const sbqa_schedule *s, const InstanceFacts &facts, hipStream_t stream, sbqa_ctx **out,
                       bool allow_resident, const uint32_t *jbits) {
    sbqa_ctx *c = new (std::nothrow) sbqa_ctx();
    if (!c) return fail(SBQA_ENOMEM, "out of host memory");
    c->N = N;
    c->R = R;
    c->runs = runs;
    c->s = *s;
    c->s.beta = c->s.alpha = nullptr;
    c->s.jp_table = nullptr;
    c->facts = facts;
    c->c0 = s->c0 > 0 ? s->c0 : (facts.rms > 0 ? 0.5 / (std::sqrt((double)N) * facts.rms) : 0.0);
    plan_layout(N, R, runs, facts, &c->L);
    build_schedule_host(s, runs, c->beta, c->alpha, c->jp_host);
    sbqa_status st = check_device(&c->device);
    if (st != SBQA_OK) { delete c; return st; }
    if (stream) c->stream = stream;
    else {
        hipError_t e = library_stream(c->device, &c->default_stream);
        if (e != hipSuccess) { delete c; return fail(SBQA_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e)); }
        c->stream = c->default_stream;
    }
    Relabelled rl;
    if (facts.path == PATH_CSR) {
        plan_reorder(J, N, s->reorder, &c->pnew);
        if (!c->pnew.empty()) {
            relabel(J, h, N, c->pnew, &rl);
            J = &rl.J;
            h = h ? rl.h.data() : nullptr;
        }
    }
    if (facts.jbits) allow_resident = false;   // the small dense loop needs J in float32
    {
        std::string why;
        const bool plan = facts.path == PATH_CSR ? resident_plan(c, J, &why) : small_plan(c, &why);
        c->resident = allow_resident && s->loop_kernel != SBQA_LOOP_STREAM && plan;
        if (!c->resident && s->loop_kernel == SBQA_LOOP_RESIDENT) {
            delete c;
            return fail(SBQA_EINVAL, "instance does not fit a resident loop: %s",
                        allow_resident ? why.c_str() : "contexts of the serving loop step one launch at a time");
        }
    }
    if (facts.path != PATH_CSR)
        set_tile(&c->L, s->dense_tile ? s->dense_tile / 64 : tune_dense_mbw(facts.path, c->L.C, c->L.Np, c->stream));
    if (facts.path != PATH_CSR) {
        c->order = ORDER_REPLICA_MAJOR;
        c->ld = c->L.Np;
    } else if (c->resident) {
        c->order = ORDER_COLBLOCK8;   // C is a multiple of 8 (R is), so Cs == C
        c->ld = c->res_rows;
    } else {
        c->order = ORDER_SPIN_MAJOR;
        c->ld = c->L.Cs;
    }
    st = ctx_upload(c, J, h, jbits);
    if (st == SBQA_OK && !c->pnew.empty()) {
        std::vector<int32_t> orig((size_t)N);
        for (int32_t i = 0; i < N; ++i) orig[(size_t)c->pnew[(size_t)i]] = i;
        hipError_t e = dalloc(c, &c->porig, (size_t)N);
        if (e == hipSuccess) e = hipMemcpyAsync(c->porig, orig.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);   // the staging vector dies here
        if (e != hipSuccess) st = fail(SBQA_EDEVICE, "relabelling: %s", hipGetErrorString(e));
    }
    if (st == SBQA_OK) {
        hipError_t e = launch_init_state(N, c->L.C, c->order, c->ld, s->seed, s->init_amp, c->porig, c->x[0], c->y,
                                         c->stream);
        if (e != hipSuccess) st = fail(SBQA_EDEVICE, "init: %s", hipGetErrorString(e));
    }
    if (st == SBQA_OK) st = rebuild_operand(c);
    if (st == SBQA_OK) st = ctx_reset_best(c);
    if (st != SBQA_OK) { delete c; return st; }
    *out = c;
    return SBQA_OK;
}

// K steps of the small dense loop in one launch (one workgroup per run);
// afterwards the fragment-tiled operand is rebuilt from the new state.
static sbqa_status ctx_step_small(sbqa_ctx *c, uint32_t K) {
    SmallArgs a;
    a.N = c->N;
    a.Np = c->L.Np;
    a.R = c->R;
    a.S = (int)c->s.steps;
    a.n0 = (int)c->step;
    a.K = (int)K;
    a.fmode = c->s.fmode;
    a.jbits = c->facts.ternary ? 1 : 0;
    a.J = c->Jsm;
    a.h = c->h32;
    a.x = c->x[c->cur];
    a.y = c->y;
    a.jp = c->jp;
    a.coefA = c->coefA;
    a.delta = c->delta_tab;
    const StepCoef k = step_coef(&c->s, c->c0, c->R, c->step);
    a.kB = k.kB;
    a.dt = k.dt;
    a.kD = k.kD;
    HIP_TRY(launch_dense_small(a, c->runs, c->stream));
    c->step += K;
    return rebuild_operand(c);
}

// K steps of the register-resident loop in one launch. A wait that timed out
// sets the error word of the readout block, which every synchronising call
// copies back and reports.
static sbqa_status ctx_step_resident(sbqa_ctx *c, uint32_t K) {
    if (c->facts.path != PATH_CSR) return ctx_step_small(c, K);
    ResidentArgs a;
    a.N = c->N;
    a.R = c->R;
    a.S = (int)c->s.steps;
    a.n0 = (int)c->step;
    a.K = (int)K;
    a.fmode = c->s.fmode;
    a.nwg = c->res_nwg;
    a.colpad = c->colpad;
    a.valpad = c->valpad;
    a.h = c->h32;
    a.x = c->x[c->cur];
    a.y = c->y;
    a.jp = c->jp;
    a.coefA = c->coefA;
    a.delta = c->delta_tab;
    const StepCoef k = step_coef(&c->s, c->c0, c->R, c->step);
    a.kB = k.kB;
    a.dt = k.dt;
    a.kD = k.kD;
    a.xpub = c->xpub;
    a.flags = c->flags;
    a.epoch_cnt = c->epoch_cnt;
    a.epoch = ++c->epoch;
    a.err = c->err;
    a.sbits = c->sbits;
    HIP_TRY(launch_csr_resident(a, c->res_D, c->stream));
    c->step += K;
    c->sbits_step = c->step;
    return SBQA_OK;
}

sbqa_status ctx_check_async(sbqa_ctx *c) {
    if (c->rhost && *reinterpret_cast<const int *>(c->rhost + (size_t)8 * c->runs))
        return fail(SBQA_EDEVICE, "resident sparse loop: a ring-neighbour wait timed out; the state is invalid");
    return SBQA_OK;
}

sbqa_status ctx_sync(sbqa_ctx *c) {
    HIP_TRY(hipMemcpyAsync(c->rhost + (size_t)8 * c->runs, c->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return ctx_check_async(c);
}

sbqa_status ctx_step(sbqa_ctx *c, uint32_t n) {
    if ((uint64_t)c->step + n > c->s.steps)
        return fail(SBQA_ESTATE, "step %u + %u exceeds the schedule of %u steps", c->step, n, c->s.steps);
    if (c->resident) {
        uint32_t left = n;
        while (left) {
            uint32_t K = left;
            if (c->s.energy_every) K = std::min(K, c->s.energy_every - c->step % c->s.energy_every);
            sbqa_status st = ctx_step_resident(c, K);
            if (st != SBQA_OK) return st;
            left -= K;
            if (c->s.energy_every && c->step % c->s.energy_every == 0) {
                st = ctx_evaluate(c);
                if (st != SBQA_OK) return st;
            }
        }
        return SBQA_OK;
    }
    for (uint32_t q = 0; q < n; ++q) {
        sbqa_status st = ctx_step_once(c);
        if (st != SBQA_OK) return st;
        if (c->s.energy_every && c->step % c->s.energy_every == 0) {
            st = ctx_evaluate(c);
            if (st != SBQA_OK) return st;
        }
    }
    return SBQA_OK;
}

// Readout: without energy tracking the best of the current state alone
// (the previous best discarded on the device, no host round trip); then the
// readout block (best energies, error word, best spins) in one copy to the
// pinned host block. Nothing waits: the results are there once the context's
// stream has passed this point.
sbqa_status ctx_readout_async(sbqa_ctx *c) {
    const bool reset = c->s.energy_every == 0;
    const bool eval = reset || c->last_eval_step != (int64_t)c->step;
    if (eval && c->rd_cnt && c->rhost_dev && c->order == ORDER_COLBLOCK8 && !c->facts.n3) {
        // resident context: energies, best update and the host block in one
        // launch (the same values as the three-launch form below)
        const int nrb = c->L.csr_nrb, rpb = (c->N + nrb - 1) / nrb;
        ReadoutFuse f;
        f.R = c->R;
        f.runs = c->runs;
        f.best_E = c->bestE;
        f.best_step = c->bestStep;
        f.best_spins = c->bestSpins;
        f.err = c->err;
        f.cnt = c->rd_cnt;
        f.host = c->rhost_dev;
        f.step = (int64_t)c->step;
        f.reset = reset ? 1 : 0;
        HIP_TRY(launch_csr_readout_colblock(c->N, c->ld, c->L.C, c->res_D, nrb, rpb, c->rcol, c->rval, c->rh,
                                            c->x[c->cur], colblock_signs(c), c->E, f, c->stream));
        c->last_eval_step = c->step;
        return SBQA_OK;
    }
    if (eval) {
        sbqa_status st = ctx_evaluate(c, reset);
        if (st != SBQA_OK) return st;
    }
    // a copy kernel right behind the readout kernels (a runtime copy started
    // 11 us after the last kernel had finished)
    if (c->rhost_dev) HIP_TRY(launch_copy_to_host(c->rdev, c->rhost_dev, c->rbytes, c->stream));
    else HIP_TRY(hipMemcpyAsync(c->rhost, c->rdev, c->rbytes, hipMemcpyDeviceToHost, c->stream));
    return SBQA_OK;
}

// The results of the last ctx_readout_async, once its work has completed.
sbqa_status ctx_readout_collect(sbqa_ctx *c, double *energies, int8_t *spins) {
    const double *bE = reinterpret_cast<const double *>(c->rhost);
    const int8_t *bS = reinterpret_cast<const int8_t *>(c->rhost + (size_t)8 * c->runs + 8);
    if (energies) std::memcpy(energies, bE, sizeof(double) * c->runs);
    if (spins) {
        if (c->pnew.empty()) std::memcpy(spins, bS, (size_t)c->runs * c->N);
        else   // back to the caller's spin order
            for (int r = 0; r < c->runs; ++r)
                for (int i = 0; i < c->N; ++i)
                    spins[(size_t)r * c->N + i] = bS[(size_t)r * c->N + c->pnew[(size_t)i]];
    }
    return ctx_check_async(c);
}

sbqa_status ctx_best(sbqa_ctx *c, double *energies, int8_t *spins) {
    sbqa_status st = ctx_readout_async(c);
    if (st != SBQA_OK) return st;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return ctx_readout_collect(c, energies, spins);
}

}  // namespace sbqa

// =========================================================================== //
//                                 C ABI                                       //
// =========================================================================== //

extern "C" {

sbqa_schedule sbqa_schedule_default(void) {
    sbqa_schedule s;
    std::memset(&s, 0, sizeof s);
    s.steps = 1000;
    s.dt = 0.5;
    s.a0 = 1.0;
    s.c0 = 0.0;
    s.fmode = SBQA_F_TERNARY;
    s.delta_max = 0.7;
    s.jp_kind = SBQA_JP_PAPER;
    s.jp_start = 0.5;
    s.jp_end = 0.0;
    s.gamma0_over_R = 1.0;
    s.beta_lo = 0.5;
    s.beta_hi = 1.5;
    s.alpha_lo = 0.5;
    s.alpha_hi = 1.0;
    s.seed = 0;
    s.init_amp = 0.1;
    s.precision = SBQA_PREC_AUTO;
    s.energy_every = 0;
    s.loop_kernel = SBQA_LOOP_AUTO;
    s.dense_tile = 0;
    s.j_packing = SBQA_JPACK_AUTO;
    s.reorder = SBQA_REORDER_AUTO;
    return s;
}

const char *sbqa_last_error(void) { return last_error(); }

sbqa_status sbqa_create(const sbqa_coupling *J, const double *h, int32_t N, int32_t R, int32_t runs,
                        const sbqa_schedule *s, sbqa_ctx **out) {
    clear_error();
    if (!out) return fail(SBQA_EINVAL, "out must be non-NULL");
    *out = nullptr;
    InstanceFacts facts;
    sbqa_status st = validate_instance(J, h, N, R, runs, s, &facts);
    if (st != SBQA_OK) return st;
    return ctx_create(J, h, N, R, runs, s, facts, nullptr, out, true);
}

sbqa_status sbqa_step(sbqa_ctx *c, uint32_t n) {
    clear_error();
    if (!c) return fail(SBQA_EINVAL, "NULL context");
    return ctx_step(c, n);
}

sbqa_status sbqa_best(sbqa_ctx *c, double *energies, int8_t *spins) {
    clear_error();
    if (!c) return fail(SBQA_EINVAL, "NULL context");
    return ctx_best(c, energies, spins);
}

sbqa_status sbqa_best_step(sbqa_ctx *c, int64_t *step_of_best) {
    clear_error();
    if (!c || !step_of_best) return fail(SBQA_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(step_of_best, c->bestStep, sizeof(int64_t) * c->runs, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SBQA_OK;
}

sbqa_status sbqa_energy(sbqa_ctx *c, const int8_t *spins, int32_t count, double *out) {
    clear_error();
    if (!c || (!spins && count) || (!out && count)) return fail(SBQA_EINVAL, "NULL argument");
    if (count < 0) return fail(SBQA_EINVAL, "count must be >= 0");
    if (count == 0) return SBQA_OK;
    const int N = c->N;
    for (int64_t q = 0; q < (int64_t)count * N; ++q)
        if (spins[q] != 1 && spins[q] != -1) return fail(SBQA_EINVAL, "spins must be +-1 (index %lld)", (long long)q);
    int8_t *ds = nullptr;
    double *E = nullptr;
    HIP_TRY(hipMalloc(&ds, (size_t)count * N));
    hipError_t e = hipMalloc(&E, sizeof(double) * count);
    if (e != hipSuccess) { (void)hipFree(ds); return fail(SBQA_ENOMEM, "hipMalloc: %s", hipGetErrorString(e)); }
    struct Guard { void *a, *b, *c2, *d; ~Guard() { (void)hipFree(a); (void)hipFree(b); (void)hipFree(c2); (void)hipFree(d); } } gd{ds, E, nullptr, nullptr};
    std::vector<int8_t> rows;
    if (!c->pnew.empty()) {   // the caller's spin order to the internal rows
        rows.resize((size_t)count * N);
        for (int32_t m = 0; m < count; ++m)
            for (int i = 0; i < N; ++i) rows[(size_t)m * N + c->pnew[(size_t)i]] = spins[(size_t)m * N + i];
    }
    HIP_TRY(hipMemcpyAsync(ds, rows.empty() ? spins : rows.data(), (size_t)count * N, hipMemcpyHostToDevice, c->stream));
    if (!rows.empty()) HIP_TRY(hipStreamSynchronize(c->stream));   // the staging vector dies at return
    double *S = nullptr, *P = nullptr;
    if (c->facts.path != PATH_CSR) {
        const EnergyGemm g = energy_gemm(c, count);
        HIP_TRY(hipMalloc(&S, sizeof(double) * g.cp * c->L.Np));
        gd.c2 = S;
        HIP_TRY(hipMalloc(&P, sizeof(double) * g.es * g.cp * c->L.Np));
        gd.d = P;
    }
    sbqa_status st = ctx_energies_dev(c, ds, count, E, S, P);
    if (st != SBQA_OK) return st;
    HIP_TRY(hipMemcpyAsync(out, E, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SBQA_OK;
}

sbqa_status sbqa_fields(sbqa_ctx *c, float *phi) {
    clear_error();
    if (!c || !phi) return fail(SBQA_EINVAL, "NULL argument");
    const int N = c->N, C = c->L.C;
    std::vector<float> buf;
    if (c->facts.path == PATH_CSR) {
        const int Cs = c->L.Cs;
        const float *xs = c->x[c->cur];
        const int8_t *gs = (const int8_t *)c->g[c->cur];
        if (c->order == ORDER_COLBLOCK8) {
            // the fields kernel gathers spin-major rows: a spin-major copy of
            // the state and its operand, and the fields, in buffers allocated
            // at the first call on a resident context
            if (!c->phi) {
                int8_t *gsm0 = nullptr;
                HIP_TRY(dalloc(c, &c->x[1 - c->cur], (size_t)N * Cs));
                HIP_TRY(dalloc(c, &gsm0, (size_t)N * Cs));
                c->g[1 - c->cur] = gsm0;
                HIP_TRY(dalloc(c, &c->phi, (size_t)N * Cs));
            }
            float *xsm = c->x[1 - c->cur];
            int8_t *gsm = (int8_t *)c->g[1 - c->cur];
            HIP_TRY(launch_state_reorder(N, C, c->order, c->ld, xs, ORDER_SPIN_MAJOR, Cs, xsm, c->stream));
            if (c->s.fmode != SBQA_F_BALLISTIC)
                HIP_TRY(launch_csr_operand(c->s.fmode, N, Cs, C, xsm, gsm, delta_at(&c->s, c->step), c->stream));
            xs = xsm;
            gs = gsm;
        }
        HIP_TRY(launch_csr_fields(c->s.fmode, N, Cs, C, c->rp, c->col, c->val, c->tri3(), xs, gs, c->phi, c->stream));
        buf.resize((size_t)N * Cs);
        HIP_TRY(hipMemcpyAsync(buf.data(), c->phi, sizeof(float) * buf.size(), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int i = 0; i < N; ++i)
            std::memcpy(phi + (size_t)i * C, buf.data() + (size_t)(c->pnew.empty() ? i : c->pnew[(size_t)i]) * Cs,
                        sizeof(float) * C);
        return SBQA_OK;
    }
    const int Np = c->L.Np;
    float *sum = nullptr;
    HIP_TRY(hipMalloc(&sum, sizeof(float) * (size_t)C * Np));
    struct G1 { void *p; ~G1() { (void)hipFree(p); } } g1{sum};
    DenseStepArgs a = dense_args(c, c->step, c->cur);
    a.phi = sum;
    HIP_TRY(launch_dense_step(c->facts.path, EPI_FIELDS, c->L.mbw, c->L.Cg, a, c->stream));
    buf.resize((size_t)C * Np);
    HIP_TRY(hipMemcpyAsync(buf.data(), sum, sizeof(float) * buf.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int i = 0; i < N; ++i)
        for (int cc = 0; cc < C; ++cc) phi[(size_t)i * C + cc] = buf[(size_t)cc * Np + i];
    return SBQA_OK;
}

sbqa_status sbqa_get_state(sbqa_ctx *c, float *x, float *y) {
    clear_error();
    if (!c) return fail(SBQA_EINVAL, "NULL context");
    const int N = c->N, C = c->L.C;
    const size_t tot = state_elems(c);
    std::vector<float> bx(tot), by(tot);
    HIP_TRY(hipMemcpyAsync(bx.data(), c->x[c->cur], sizeof(float) * tot, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(by.data(), c->y, sizeof(float) * tot, hipMemcpyDeviceToHost, c->stream));
    {
        sbqa_status e = ctx_sync(c);
        if (e != SBQA_OK) return e;
    }
    for (int i = 0; i < N; ++i) {
        const int row = c->pnew.empty() ? i : c->pnew[(size_t)i];   // internal row of spin i
        for (int cc = 0; cc < C; ++cc) {
            const int64_t o = state_off(c->order, c->ld, row, cc);
            if (x) x[(size_t)i * C + cc] = bx[(size_t)o];
            if (y) y[(size_t)i * C + cc] = by[(size_t)o];
        }
    }
    return SBQA_OK;
}

sbqa_status sbqa_set_state(sbqa_ctx *c, const float *x, const float *y) {
    clear_error();
    if (!c || !x || !y) return fail(SBQA_EINVAL, "NULL argument");
    const int N = c->N, C = c->L.C;
    const size_t tot = state_elems(c);
    for (size_t q = 0; q < (size_t)N * C; ++q)
        if (!std::isfinite(x[q]) || !std::isfinite(y[q]) || std::fabs(x[q]) > 1.0f)
            return fail(SBQA_EINVAL, "state must be finite with |x| <= 1 (index %zu)", q);
    std::vector<float> bx(tot, 0.0f), by(tot, 0.0f);   // padding rows and columns stay zero
    for (int i = 0; i < N; ++i) {
        const int row = c->pnew.empty() ? i : c->pnew[(size_t)i];   // internal row of spin i
        for (int cc = 0; cc < C; ++cc) {
            const int64_t o = state_off(c->order, c->ld, row, cc);
            bx[(size_t)o] = x[(size_t)i * C + cc];
            by[(size_t)o] = y[(size_t)i * C + cc];
        }
    }
    HIP_TRY(hipMemcpyAsync(c->x[c->cur], bx.data(), sizeof(float) * tot, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->y, by.data(), sizeof(float) * tot, hipMemcpyHostToDevice, c->stream));
    c->sbits_step = -1;
    sbqa_status st = rebuild_operand(c);
    if (st != SBQA_OK) return st;
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->last_eval_step = -1;
    return SBQA_OK;
}

sbqa_status sbqa_run_params(sbqa_ctx *c, double *beta, double *alpha) {
    clear_error();
    if (!c) return fail(SBQA_EINVAL, "NULL context");
    if (beta) std::memcpy(beta, c->beta.data(), sizeof(double) * c->runs);
    if (alpha) std::memcpy(alpha, c->alpha.data(), sizeof(double) * c->runs);
    return SBQA_OK;
}

sbqa_status sbqa_jperp_table(sbqa_ctx *c, float *jp) {
    clear_error();
    if (!c || !jp) return fail(SBQA_EINVAL, "NULL argument");
    std::memcpy(jp, c->jp_host.data(), sizeof(float) * c->jp_host.size());
    return SBQA_OK;
}

sbqa_status sbqa_set_stream(sbqa_ctx *c, void *hip_stream) {
    clear_error();
    if (!c) return fail(SBQA_EINVAL, "NULL context");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->stream = hip_stream ? (hipStream_t)hip_stream : c->default_stream;
    if (!c->stream) return fail(SBQA_ESTATE, "context has no default stream");
    return SBQA_OK;
}

sbqa_status sbqa_info(sbqa_ctx *c, sbqa_info_t *info) {
    clear_error();
    if (!c || !info) return fail(SBQA_EINVAL, "NULL argument");
    info->N = c->N;
    info->R = c->R;
    info->runs = c->runs;
    info->steps = c->s.steps;
    info->step = c->step;
    info->path = c->facts.path;
    info->fmode = c->s.fmode;
    info->c0 = c->c0;
    info->j_integral = c->facts.integral ? 1 : 0;
    info->device_bytes = c->bytes;
    info->resident = c->resident ? 1 : 0;
    info->tile_cols = c->facts.path == PATH_CSR ? 0 : 64 * c->L.mbw;
    info->reordered = c->pnew.empty() ? 0 : 1;
    return SBQA_OK;
}

sbqa_status sbqa_sync(sbqa_ctx *c) {
    clear_error();
    if (!c) return fail(SBQA_EINVAL, "NULL context");
    return ctx_sync(c);
}

sbqa_status sbqa_inject_wait_timeout(sbqa_ctx *c) {
    clear_error();
    if (!c) return fail(SBQA_EINVAL, "NULL context");
    if (!c->resident || c->facts.path != PATH_CSR || !c->err)
        return fail(SBQA_EINVAL, "the context does not run the resident sparse loop");
    static const int timed_out = 1;   // the value a timed-out wait stores
    HIP_TRY(hipMemcpyAsync(c->err, &timed_out, sizeof(int), hipMemcpyHostToDevice, c->stream));
    return SBQA_OK;
}

void sbqa_destroy(sbqa_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"
