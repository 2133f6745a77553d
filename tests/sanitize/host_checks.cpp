// Host-side checks of the SBQA runtime, built with the host part of every
// source instrumented by AddressSanitizer + UndefinedBehaviorSanitizer, or by
// ThreadSanitizer (paper_2604_01050_amd/build.py, build_sanitized). This
// translation unit includes the runtime's own source so that it can call the
// internal steps that run before any device work:
//   * validation of CSR and dense couplings, fuzzed with malformed structures
//     held in exactly sized heap buffers (an out-of-bounds read is reported);
//   * the host schedule (Eq. 5 per run, linear, tables);
//   * the reverse Cuthill-McKee relabelling and the relabelled copy (every row
//     keeps its couplings in the given order, triples and fields follow);
//   * the argument paths of the C ABI and of the serving interface.
// With a GPU present it also runs a serving stream submitted and polled from
// several client threads, so that the scheduler and creator threads run under
// ThreadSanitizer. Prints "host checks passed" and returns 0 on success.
#include "../../paper_2604_01050_amd/csrc/sbqa_api.cpp"

#include <unistd.h>

#include <atomic>
#include <cstdio>
#include <random>
#include <thread>

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                         \
    do {                                                         \
        if (!(cond)) {                                           \
            std::fprintf(stderr, "CHECK failed %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                   \
            std::fprintf(stderr, "\n");                          \
            ++g_fail;                                            \
        }                                                        \
    } while (0)

struct Csr {
    int32_t N = 0;
    std::vector<int32_t> rp, col;
    std::vector<double> val;
};

// Random symmetric sparse couplings with sorted columns (a d-regular-like graph).
Csr random_csr(std::mt19937_64 &g, int32_t N, int deg) {
    std::vector<std::vector<std::pair<int32_t, double>>> rows((size_t)N);
    std::uniform_int_distribution<int32_t> pick(0, N - 1);
    std::normal_distribution<double> w(0.0, 1.0);
    for (int32_t i = 0; i < N; ++i)
        for (int e = 0; e < deg / 2; ++e) {
            const int32_t j = pick(g);
            if (j == i) continue;
            bool dup = false;
            for (auto &pr : rows[(size_t)i]) dup |= pr.first == j;
            if (dup) continue;
            const double v = w(g);
            rows[(size_t)i].push_back({j, v});
            rows[(size_t)j].push_back({i, v});
        }
    Csr c;
    c.N = N;
    c.rp.assign((size_t)N + 1, 0);
    for (int32_t i = 0; i < N; ++i) {
        std::sort(rows[(size_t)i].begin(), rows[(size_t)i].end());
        c.rp[(size_t)i + 1] = c.rp[(size_t)i] + (int32_t)rows[(size_t)i].size();
        for (auto &pr : rows[(size_t)i]) {
            c.col.push_back(pr.first);
            c.val.push_back(pr.second);
        }
    }
    return c;
}

sbqa_coupling coupling_of(const Csr &c) {
    sbqa_coupling J{};
    J.row_ptr = c.rp.data();
    J.col = c.col.data();
    J.val = c.val.data();
    J.nnz = (int64_t)c.col.size();
    return J;
}

sbqa_schedule sched(uint32_t steps) {
    sbqa_schedule s = sbqa_schedule_default();
    s.steps = steps;
    return s;
}

void check_validation(std::mt19937_64 &g) {
    const sbqa_schedule s = sched(20);
    for (int trial = 0; trial < 300; ++trial) {
        const int32_t N = 2 + (int32_t)(g() % 300);
        Csr c = random_csr(g, N, 2 + (int)(g() % 6));
        InstanceFacts f;
        sbqa_coupling J = coupling_of(c);
        CHECK(validate_instance(&J, nullptr, N, 8, 2, &s, &f) == SBQA_OK, "valid CSR rejected: %s", last_error());
        // one mutation; the buffers keep their exact sizes
        const int kind = (int)(g() % 7);
        const size_t nnz = c.col.size();
        bool invalid = true;
        switch (kind) {
            case 0: c.rp[1 + g() % (size_t)N] = (int32_t)(nnz + 1 + g() % 1000); break;   // past nnz
            case 1: c.rp[1 + g() % (size_t)N] = -(int32_t)(1 + g() % 5); break;              // negative
            case 2:
                if (!nnz) { invalid = false; break; }
                c.col[g() % nnz] = (g() & 1) ? N + (int32_t)(g() % 50) : -1;
                break;
            case 3:
                if (!nnz) { invalid = false; break; }
                c.val[g() % nnz] = std::numeric_limits<double>::quiet_NaN();
                break;
            case 4:
                if (!nnz) { invalid = false; break; }
                c.val[g() % nnz] += 0.5;   // asymmetric
                break;
            case 5:
                c.rp[(size_t)N] = (int32_t)nnz + 3;   // row_ptr[N] != nnz
                break;
            default: {
                if (nnz < 2) { invalid = false; break; }
                const size_t p = g() % (nnz - 1);
                std::swap(c.col[p], c.col[p + 1]);   // unsorted (or a no-op across rows)
                invalid = false;                      // may stay valid when p ends a row
            }
        }
        J = coupling_of(c);
        J.nnz = (int64_t)nnz;
        const sbqa_status st = validate_instance(&J, nullptr, N, 8, 2, &s, &f);
        if (invalid) CHECK(st == SBQA_EINVAL, "mutation %d accepted (N=%d)", kind, N);
    }
    // dense: non-zero diagonal, NaN, asymmetric; all-zero J; N = 1
    for (int trial = 0; trial < 40; ++trial) {
        const int32_t N = 1 + (int32_t)(g() % 70);
        std::vector<double> A((size_t)N * N, 0.0);
        for (int32_t i = 0; i < N; ++i)
            for (int32_t j = 0; j < i; ++j) A[(size_t)i * N + j] = A[(size_t)j * N + i] = (g() & 1) ? 1.0 : -1.0;
        sbqa_coupling J{};
        J.dense = A.data();
        InstanceFacts f;
        CHECK(validate_instance(&J, nullptr, N, 4, 3, &s, &f) == SBQA_OK, "valid dense rejected: %s", last_error());
        if (N > 1) {
            const size_t i = g() % (size_t)N, j = (i + 1) % (size_t)N;
            const int kind = trial % 3;
            if (kind == 0) A[i * N + i] = 2.0;
            else if (kind == 1) A[i * N + j] = std::numeric_limits<double>::infinity();
            else A[i * N + j] = 5.0;
            CHECK(validate_instance(&J, nullptr, N, 4, 3, &s, &f) == SBQA_EINVAL, "dense mutation %d accepted", kind);
        }
    }
}

void check_schedule(std::mt19937_64 &g) {
    for (int trial = 0; trial < 50; ++trial) {
        sbqa_schedule s = sched(1 + (uint32_t)(g() % 500));
        const int runs = 1 + (int)(g() % 9);
        s.jp_kind = (sbqa_jpkind)(g() % 2);
        s.seed = g();
        s.gamma0_over_R = 0.05 + (double)(g() % 100);
        std::vector<double> beta, alpha;
        std::vector<float> jp;
        build_schedule_host(&s, runs, beta, alpha, jp);
        CHECK(jp.size() == (size_t)runs * s.steps, "table size");
        for (float v : jp) CHECK(std::isfinite(v) && v >= 0.0f, "J_perp %g", (double)v);
        for (int r = 0; r < runs; ++r)
            CHECK(beta[(size_t)r] >= s.beta_lo && beta[(size_t)r] <= s.beta_hi && alpha[(size_t)r] >= s.alpha_lo &&
                      alpha[(size_t)r] <= s.alpha_hi, "beta/alpha out of range");
    }
}

void check_relabel(std::mt19937_64 &g) {
    for (int trial = 0; trial < 40; ++trial) {
        const int32_t N = 3 + (int32_t)(g() % 3000);
        Csr c = random_csr(g, N, 2 + (int)(g() % 6));
        std::vector<int32_t> tri;
        std::vector<double> K;
        const int n3 = (int)(g() % 20);
        for (int t = 0; t < n3; ++t) {
            const int32_t a = (int32_t)(g() % N), b = (int32_t)(g() % N), d = (int32_t)(g() % N);
            if (a == b || a == d || b == d) continue;
            tri.insert(tri.end(), {a, b, d});
            K.push_back(1.0 + t);
        }
        std::vector<double> h((size_t)N);
        for (int32_t i = 0; i < N; ++i) h[(size_t)i] = 0.01 * i;
        sbqa_coupling J = coupling_of(c);
        J.n3 = (int64_t)K.size();
        J.tri = J.n3 ? tri.data() : nullptr;
        J.K = J.n3 ? K.data() : nullptr;
        std::vector<int32_t> pnew;
        plan_reorder(&J, N, SBQA_REORDER_ON, &pnew);
        if (J.nnz == 0 && J.n3 == 0) {
            CHECK(pnew.empty(), "relabelled an instance without couplings");
            continue;
        }
        CHECK((int32_t)pnew.size() == N, "permutation size");
        std::vector<int32_t> seen((size_t)N, 0);
        for (int32_t v : pnew) {
            CHECK(v >= 0 && v < N, "label out of range");
            if (v >= 0 && v < N) ++seen[(size_t)v];
        }
        for (int32_t k : seen) CHECK(k == 1, "not a permutation");
        Relabelled rl;
        relabel(&J, h.data(), N, pnew, &rl);
        for (int32_t i = 0; i < N; ++i) {
            const int32_t k = pnew[(size_t)i];
            CHECK(rl.rp[(size_t)k + 1] - rl.rp[(size_t)k] == c.rp[(size_t)i + 1] - c.rp[(size_t)i], "row length");
            for (int32_t q = 0; q < c.rp[(size_t)i + 1] - c.rp[(size_t)i]; ++q) {
                CHECK(rl.col[(size_t)(rl.rp[(size_t)k] + q)] == pnew[(size_t)c.col[(size_t)(c.rp[(size_t)i] + q)]], "column");
                CHECK(rl.val[(size_t)(rl.rp[(size_t)k] + q)] == c.val[(size_t)(c.rp[(size_t)i] + q)], "weight");
            }
            CHECK(rl.h[(size_t)k] == h[(size_t)i], "field");
        }
        for (size_t q = 0; q < tri.size(); ++q) CHECK(rl.tri[q] == pnew[(size_t)tri[q]], "triple");
    }
}

void check_abi_arguments() {
    sbqa_ctx *ctx = nullptr;
    CHECK(sbqa_create(nullptr, nullptr, 4, 1, 1, nullptr, &ctx) == SBQA_EINVAL, "create(NULL)");
    CHECK(sbqa_step(nullptr, 1) == SBQA_EINVAL, "step(NULL)");
    CHECK(sbqa_best(nullptr, nullptr, nullptr) == SBQA_EINVAL, "best(NULL)");
    CHECK(sbqa_energy_noalloc(nullptr, nullptr, 1, nullptr) == SBQA_EINVAL, "energy_noalloc(NULL)");
    sbqa_server *srv = nullptr;
    CHECK(sbqa_server_create(0, 4, &srv) == SBQA_EINVAL, "server budget 0");
    CHECK(sbqa_server_create(1 << 20, 0, &srv) == SBQA_EINVAL, "server slots 0");
    uint64_t t = 0;
    CHECK(sbqa_submit(nullptr, nullptr, nullptr, 4, 1, 1, nullptr, &t) == SBQA_EINVAL, "submit(NULL)");
    CHECK(sbqa_poll(nullptr, 1, nullptr, nullptr, nullptr) == SBQA_EINVAL, "poll(NULL)");
}

// Serving stream from several client threads (needs a GPU).
void check_server_threads(std::mt19937_64 &g) {
    sbqa_server *srv = nullptr;
    if (sbqa_server_create((size_t)256 << 20, 3, &srv) != SBQA_OK) {
        std::fprintf(stderr, "server_create: %s\n", sbqa_last_error());
        ++g_fail;
        return;
    }
    struct Item {
        Csr csr;
        std::vector<double> dense;
        int32_t N;
    };
    std::vector<Item> items;
    for (int q = 0; q < 12; ++q) {
        Item it;
        it.N = 100 + (int32_t)(g() % 300);
        if (q % 2) {
            it.csr = random_csr(g, it.N, 4);
        } else {
            it.dense.assign((size_t)it.N * it.N, 0.0);
            for (int32_t i = 0; i < it.N; ++i)
                for (int32_t j = 0; j < i; ++j)
                    it.dense[(size_t)i * it.N + j] = it.dense[(size_t)j * it.N + i] = (g() & 1) ? 1.0 : -1.0;
        }
        items.push_back(std::move(it));
    }
    std::atomic<int> done{0}, bad{0};
    auto client = [&](int c) {
        for (size_t q = (size_t)c; q < items.size(); q += 3) {
            const Item &it = items[q];
            sbqa_coupling J = it.dense.empty() ? coupling_of(it.csr) : sbqa_coupling{};
            if (!it.dense.empty()) J.dense = it.dense.data();
            sbqa_schedule s = sched(300);
            s.seed = q;
            uint64_t ticket = 0;
            if (sbqa_submit(srv, &J, nullptr, it.N, 8, 2, &s, &ticket) != SBQA_OK) {
                ++bad;
                continue;
            }
            std::vector<double> E(2);
            std::vector<int8_t> spins((size_t)2 * it.N);
            double lat = 0;
            sbqa_status st;
            const auto t0 = std::chrono::steady_clock::now();
            while ((st = sbqa_poll(srv, ticket, E.data(), spins.data(), &lat)) == SBQA_EAGAIN &&
                   std::chrono::steady_clock::now() - t0 < std::chrono::seconds(60))
                std::this_thread::sleep_for(std::chrono::milliseconds(1));
            if (st != SBQA_OK || !std::isfinite(E[0]) || !std::isfinite(E[1])) ++bad;
            ++done;
        }
    };
    std::vector<std::thread> th;
    for (int c = 0; c < 3; ++c) th.emplace_back(client, c);
    for (auto &x : th) x.join();
    sbqa_server_destroy(srv);
    CHECK(done == (int)items.size() && bad == 0, "serving: %d done, %d failed", done.load(), bad.load());
    std::printf("serving: %d instances submitted and polled from 3 client threads, %d failed\n", done.load(), bad.load());
}

}  // namespace

// LeakSanitizer's check, present only in address-sanitized builds.
extern "C" void __lsan_do_leak_check(void) __attribute__((weak));

int main() {
    std::setvbuf(stdout, nullptr, _IONBF, 0);   // a sanitizer's exit-time report must not swallow the output
    std::mt19937_64 g(20261203);
    check_validation(g);
    check_schedule(g);
    check_relabel(g);
    check_abi_arguments();
    int ndev = 0;
    const hipError_t de = hipGetDeviceCount(&ndev);
    (void)hipGetLastError();
    if (de == hipSuccess && ndev > 0) check_server_threads(g);
    else std::printf("no GPU (%s): serving threads not exercised\n", hipGetErrorString(de));
    const int rc = g_fail ? 1 : 0;
    if (g_fail) std::printf("host checks FAILED (%d)\n", g_fail);
    else std::printf("host checks passed\n");
    // The leak check runs here, then the process ends without running the
    // ROCm runtime's static destructors: under AddressSanitizer their
    // teardown of the sanitizer's device-allocator hooks fails an internal
    // check of the sanitizer runtime once a GPU has been used.
    if (__lsan_do_leak_check) __lsan_do_leak_check();
    std::fflush(stdout);
    std::fflush(stderr);
    _exit(rc);
}
