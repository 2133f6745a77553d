// Solver context of the SBQA library (host side) and the internal entry points
// shared by the C ABI (sbqa_api.cpp) and the serving loop (sbqa_serve.cpp).
#pragma once

#include "../../include/sbqa.h"
#include "sbqa_internal.h"

#include <string>
#include <vector>

namespace sbqa {

// What validation learned about an instance.
struct InstanceFacts {
    bool dense = true;
    bool integral = false;   // every J_ij and h_i is an integer
    bool ternary = false;    // every J_ij in {-1, 0, +1}
    bool int8 = false;       // every J_ij an integer in [-127, 127]
    bool pm1 = false;        // every off-diagonal J_ij in {-1, +1} (dense)
    int64_t n3 = 0;          // three-body terms (CSR)
    double rms = 0.0;        // rms of the N(N-1) off-diagonal couplings
    int64_t nnz = 0;
    Path path = PATH_F32;
    // dense +-1 J handed over as row-major sign bits (the serving loop packs
    // them on the host): the bit-packed contraction copy is built from them
    // and no float64 copy of J is kept (integer J: the readout energies run
    // on MFMA), so sbqa_energy is not available on such a context
    bool jbits = false;
};
// The readout energies of these paths are exact MFMA contractions (no
// float64 copy of J or energy GEMM buffers needed for them).
constexpr bool path_energy_mfma(Path p) {
    return p == PATH_FP8 || p == PATH_FP8PK || p == PATH_I8 || p == PATH_FP4 || p == PATH_FP4PK;
}
// Row-major sign bits of a dense +-1 J (InstanceFacts::jbits), ceil(N/32)
// words per row; parallel over row blocks for large N.
void pack_sign_bits(const double *J, int32_t N, std::vector<uint32_t> *bits);

// Device geometry of a context.
struct Layout {
    int C = 0;        // runs * R
    int Np = 0;       // N padded to dense_pad(path) (dense)
    int Cp = 0;       // C padded to GEMM_BM (rows of the fp64 energy GEMM)
    int Cg = 0;       // C padded to 64 * mbw (rows of the contraction operand)
    int mbw = 1;      // m-blocks per wave of the dense step
    int nkc = 0;      // K chunks of 128 bytes per operand row (dense)
    int Cs = 0;       // C padded to 4 (CSR row stride)
    int esplits = 1;  // K splits of the fp64 energy GEMM
    int csr_nrb = 0;  // row blocks of the CSR energy reduction
    size_t bytes = 0; // device bytes (without the schedule table)
};

sbqa_status fail(sbqa_status st, const char *fmt, ...);
void clear_error();
const char *last_error();

sbqa_status validate_instance(const sbqa_coupling *J, const double *h, int32_t N, int32_t R, int32_t runs,
                              const sbqa_schedule *s, InstanceFacts *facts);
void plan_layout(int32_t N, int32_t R, int32_t runs, const InstanceFacts &f, Layout *L);
size_t instance_bytes(int32_t N, int32_t R, int32_t runs, const InstanceFacts &f, uint32_t steps);
StepCoef step_coef(const sbqa_schedule *s, double c0, int R, uint32_t n);

// allow_resident: false for contexts that share the GPU with other work (the
// resident loop needs all its workgroups co-resident).
// jbits: the sign bits of a dense J when facts.jbits (J->dense is then unused).
sbqa_status ctx_create(const sbqa_coupling *J, const double *h, int32_t N, int32_t R, int32_t runs,
                       const sbqa_schedule *s, const InstanceFacts &facts, hipStream_t stream, sbqa_ctx **out,
                       bool allow_resident, const uint32_t *jbits = nullptr);
sbqa_status ctx_step(sbqa_ctx *c, uint32_t n);
sbqa_status ctx_step_once(sbqa_ctx *c);
sbqa_status ctx_best(sbqa_ctx *c, double *energies, int8_t *spins);
// ctx_best in two halves: enqueue the readout (no wait), then, once the
// context's stream has passed it, copy the results out.
sbqa_status ctx_readout_async(sbqa_ctx *c);
sbqa_status ctx_readout_collect(sbqa_ctx *c, double *energies, int8_t *spins);
sbqa_status ctx_check_async(sbqa_ctx *c);  // after a readout copy and a stream synchronisation
sbqa_status ctx_sync(sbqa_ctx *c);         // fetch the error word, synchronise, check it
// energies of the current state -> best tracking (reset: the previous best is discarded)
sbqa_status ctx_evaluate(sbqa_ctx *c, bool reset = false);
// Energies of count spin rows already on the device in the internal spin
// order (ds [count][N] int8 +-1) into E [count], on the context's stream.
// Dense couplings need float64 scratch S [cp][Np] and P [es][cp][Np] with the
// sizes energy_gemm gives (the GEMM's K splits follow the shape, so every
// caller sums in the same order); CSR couplings need none (S, P unused).
struct EnergyGemm {
    int cp = 0;   // count padded to GEMM_BM
    int es = 1;   // K splits
};
EnergyGemm energy_gemm(const sbqa_ctx *c, int count);
sbqa_status ctx_energies_dev(sbqa_ctx *c, const int8_t *ds, int32_t count, double *E, double *S, double *P);

}  // namespace sbqa

struct sbqa_ctx {
    int N = 0, R = 0, runs = 0;
    sbqa_schedule s{};                 // copy; borrowed pointers cleared
    sbqa::InstanceFacts facts;
    sbqa::Layout L;
    std::vector<double> beta, alpha;   // per-run (Sec. II.B)
    std::vector<float> jp_host;        // J_perp[r][n], run-major
    double c0 = 0.0;
    uint32_t step = 0;
    int64_t last_eval_step = -1;
    int device = 0;
    // default_stream: the library's stream of the device (shared by the
    // contexts given no stream, never destroyed); stream: where this
    // context's work is issued
    hipStream_t default_stream = nullptr, stream = nullptr;
    size_t bytes = 0;
    std::vector<void *> allocs;
    bool has_h = false;

    // state (dense: [C][Np] replica-major; CSR: [N][Cs] spin-major, or
    // column-block-major [C/8][rows][8] for the register-resident loop);
    // element (i, c) at state_off(order, ld, i, c)
    int order = 0, ld = 0;
    float *x[2] = {nullptr, nullptr};
    float *y = nullptr;
    int cur = 0;
    // operand f(X), ping-pong with x: dense fragment-tiled, CSR int8 [N][Cs]
    // (the resident CSR loop builds its own from x at each launch)
    void *g[2] = {nullptr, nullptr};
    void *g_lo[2] = {nullptr, nullptr}; // bf16 low part (BF16X3)
    float *phi = nullptr;               // CSR fields hook [N][Cs]
    void *Jd = nullptr, *Jd_lo = nullptr;  // dense J in contraction precision, fragment-tiled
    double *J64 = nullptr;              // dense J in float64 (energies)
    int32_t *rp = nullptr, *col = nullptr;
    float *val = nullptr;
    double *val64 = nullptr;
    int32_t *t3ptr = nullptr, *t3ab = nullptr;   // three-body terms per member spin (Tri3)
    float *t3k = nullptr;
    double *t3k64 = nullptr;
    sbqa::Tri3 tri3() const {
        sbqa::Tri3 t;
        if (t3ptr) { t.ptr = t3ptr; t.ab = t3ab; t.k = t3k; t.k64 = t3k64; }
        return t;
    }
    float *h32 = nullptr;
    double *h64 = nullptr;
    float *jp = nullptr;                // device J_perp table [runs][steps]
    double *S64 = nullptr, *phis64 = nullptr;
    double *csr_partial = nullptr;
    double *E = nullptr;
    int64_t *bestStep = nullptr;
    int *bsel = nullptr;                // [runs] winning replica of a readout (N > BEST_SPLIT_N)
    // readout block, one device allocation copied to the host in one piece:
    // best energies [runs] float64, the error word of the resident loop (8
    // bytes), best spins [runs][N] int8; rhost is its pinned, coherent host
    // copy and rhost_dev the device address of rhost (a copy kernel writes
    // it; nullptr: hipMemcpyAsync does)
    uint8_t *rdev = nullptr, *rhost = nullptr, *rhost_dev = nullptr;
    size_t rbytes = 0;
    double *bestE = nullptr;
    int *err = nullptr;                 // ring-neighbour wait timeouts (resident loop)
    int8_t *bestSpins = nullptr;

    // resident loops: register-resident CSR loop (kernels_csr.hip) or the
    // small dense loop (kernels_small.hip)
    bool resident = false;
    float *Jsm = nullptr;               // small dense loop: J float32 [N][N]
    int res_D = 0, res_rows = 0, res_nwg = 0;
    int32_t *colpad = nullptr;          // [rows][D]
    std::vector<int32_t> pnew;          // CSR spins relabelled: row of the caller's spin i (empty: identity)
    int32_t *porig = nullptr;           // [N] the caller's spin index of each row (relabelled only)
    float *valpad = nullptr;            // [D][rows]
    // readout energies of the resident loop: the couplings grouped by the
    // energy row blocks, row block innermost (launch_csr_energy_colblock)
    int32_t *rcol = nullptr;            // [RS][D][nrb]
    double *rval = nullptr, *rh = nullptr;   // [RS][D][nrb], [RS][nrb]
    float *coefA = nullptr;             // [S]
    float *delta_tab = nullptr;         // [S+1]
    float *xpub = nullptr;              // [2][nwg][2][rows] published edge columns
    // sign bytes of the state the resident loop left ([nwg][rows], bit k: x
    // of the block's column k is negative), valid while sbits_step == step
    uint8_t *sbits = nullptr;
    int64_t sbits_step = -1;
    // per-run arrival counters of the one-launch readout of a resident
    // context (launch_csr_readout_colblock), zero between launches
    int *rd_cnt = nullptr;
    int *flags = nullptr, *epoch_cnt = nullptr;
    int epoch = 0;

    ~sbqa_ctx();
};
