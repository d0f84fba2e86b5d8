// Host-side check of the C ABI, meant to be built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code only (device code is unchanged).
//
// Without a GPU it drives every validation and error path the host code has:
// status strings, each rejected parameter, ensemble consistency, null contexts
// and null arguments.  With a GPU it also runs a small FCC box and a 3-box
// ensemble through every entry point: state in and out, cells, lists, forces,
// steps (eager and captured), energies and their series, pressure, thermostat,
// rescaling, the autotuner with a cache file (timed, then read back), both
// bubble analyses and the statistics.  Exit status 0 when every check holds.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#include "md.h"

namespace {

int g_fail = 0;

#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            std::fprintf(stderr, "host_check: %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++g_fail;                                                                 \
        }                                                                             \
    } while (0)

#define OK(call)                                                                                 \
    do {                                                                                         \
        const md_status s_ = (call);                                                             \
        if (s_ != MD_OK) {                                                                       \
            std::fprintf(stderr, "host_check: %s:%d: %s -> %s\n", __FILE__, __LINE__, #call,     \
                         md_status_str(s_));                                                     \
            ++g_fail;                                                                            \
        }                                                                                        \
    } while (0)

md_params base(int64_t n, double L) {
    md_params p;
    std::memset(&p, 0, sizeof p);
    p.n = n;
    p.box[0] = p.box[1] = p.box[2] = L;
    p.rc = 2.5;
    p.skin = 0.3;
    p.dt = 0.005;
    p.mass = 1.0;
    p.precision = MD_PREC_FP64;
    p.cutoff = MD_CUT_EQ1;
    p.rebuild = MD_REBUILD_DUTC;
    return p;
}

void host_only_checks() {
    CHECK(std::strcmp(md_status_str(MD_OK), "MD_OK") == 0);
    CHECK(std::strcmp(md_status_str(MD_ELIST), "MD_ELIST") == 0);
    CHECK(std::strcmp(md_status_str((md_status)-99), "MD_UNKNOWN") == 0);
    CHECK(std::strcmp(md_status_str((md_status)5), "MD_UNKNOWN") == 0);
    CHECK(md_last_error(nullptr) != nullptr);

    const std::vector<std::function<void(md_params&)>> bad = {
        [](md_params& p) { p.n = 1; },
        [](md_params& p) { p.rc = 0.0; },
        [](md_params& p) { p.rc = NAN; },
        [](md_params& p) { p.skin = -0.1; },
        [](md_params& p) { p.dt = 0.0; },
        [](md_params& p) { p.mass = -1.0; },
        [](md_params& p) { p.box[0] = 8.3; },
        [](md_params& p) { p.box[1] = INFINITY; },
        [](md_params& p) { p.box[2] = 3000.0; },
        [](md_params& p) { p.precision = 7; },
        [](md_params& p) { p.cutoff = 9; },
        [](md_params& p) { p.rebuild = 5; },
        [](md_params& p) { p.flags = 1u << 7; },
        [](md_params& p) { p.flags = MD_F_TILE_ON | MD_F_TILE_OFF; },
        [](md_params& p) { p.flags = MD_F_FAST_RCP; p.precision = MD_PREC_FP32_MIXED; },
        [](md_params& p) { p.flags = MD_F_HALF_LIST | MD_F_VERIFY_LIST; },
        [](md_params& p) { p.flags = MD_F_HALF_LIST; p.threads_per_key = 2; },
        [](md_params& p) { p.threads_per_key = 3; },
        [](md_params& p) { p.list_cap = -1; },
        [](md_params& p) { p.list_cap = 5000; },
        [](md_params& p) { p.cell_scale = 0.5; },
        [](md_params& p) { p.cell_scale = NAN; },
        [](md_params& p) { p.reserved[4] = 1; },
        [](md_params& p) { p.n = (1ll << 27) + 1; p.box[0] = p.box[1] = p.box[2] = 400.0; },
    };
    for (const auto& f : bad) {
        md_params p = base(4000, 20.0);
        f(p);
        md_ctx* c = reinterpret_cast<md_ctx*>(&p);  // must come back NULL
        CHECK(md_create(&p, nullptr, &c) == MD_EINVAL);
        CHECK(c == nullptr);
        CHECK(std::strlen(md_last_error(nullptr)) > 0);
    }
    md_ctx* c = nullptr;
    md_params two[2] = {base(4000, 20.0), base(2000, 16.0)};
    CHECK(md_batch_create(two, 0, nullptr, &c) == MD_EINVAL && c == nullptr);
    CHECK(md_batch_create(nullptr, 2, nullptr, &c) == MD_EINVAL && c == nullptr);
    CHECK(md_create(nullptr, nullptr, &c) == MD_EINVAL && c == nullptr);
    two[1].rc = 3.0;
    CHECK(md_batch_create(two, 2, nullptr, &c) == MD_EINVAL && c == nullptr);
    two[1] = base(2000, 16.0);
    two[1].cell_scale = 1.2;
    CHECK(md_batch_create(two, 2, nullptr, &c) == MD_EINVAL && c == nullptr);

    // null contexts
    double x = 0.0;
    int32_t k = 0;
    int64_t t = 0;
    md_stats st;
    md_bubble_info bi;
    CHECK(md_destroy(nullptr) == MD_OK);
    CHECK(md_set_state(nullptr, nullptr, nullptr) == MD_EINVAL);
    CHECK(md_get_state(nullptr, nullptr, nullptr) == MD_EINVAL);
    CHECK(md_rescale_box(nullptr, 1.1) == MD_EINVAL);
    CHECK(md_scale_velocities(nullptr, &x) == MD_EINVAL);
    CHECK(md_build_cells(nullptr) == MD_EINVAL);
    CHECK(md_build_neighbors(nullptr) == MD_EINVAL);
    CHECK(md_compute_forces(nullptr, nullptr) == MD_EINVAL);
    CHECK(md_step(nullptr, 1, 0) == MD_EINVAL);
    CHECK(md_energy(nullptr, &x, &x) == MD_EINVAL);
    CHECK(md_batch_energy(nullptr, &x, &x) == MD_EINVAL);
    CHECK(md_energy_series(nullptr, &x, &x, 1, &k) == MD_EINVAL);
    CHECK(md_observable_series(nullptr, &x, &x, 1, &k) == MD_EINVAL);
    CHECK(md_pressure(nullptr, &x) == MD_EINVAL);
    CHECK(md_set_thermostat(nullptr, &x, 0.5) == MD_EINVAL);
    CHECK(md_get_thermostat(nullptr, &x, &x) == MD_EINVAL);
    CHECK(md_bubbles(nullptr, 0, 3.0, 0.2, nullptr, nullptr, nullptr, nullptr, 0, &bi) == MD_EINVAL);
    CHECK(md_bubbles_noalloc(nullptr, 0, 3.0, 0.2, nullptr, nullptr, nullptr, nullptr, 0, &bi) == MD_EINVAL);
    CHECK(md_get_cells(nullptr, nullptr, nullptr) == MD_EINVAL);
    CHECK(md_get_neighbors(nullptr, nullptr, nullptr, 0, &t) == MD_EINVAL);
    CHECK(md_get_stats(nullptr, &st) == MD_EINVAL);
    CHECK(md_set_timing(nullptr, 1) == MD_EINVAL);
    CHECK(md_autotune(nullptr, nullptr) == MD_EINVAL);
}

// FCC lattice of ncell^3 cubes of side a, velocities from a fixed pattern with
// zero total momentum.
void fcc(int ncell, double a, std::vector<double>& q, std::vector<double>& v) {
    static const double basis[4][3] = {{0, 0, 0}, {0.5, 0.5, 0}, {0.5, 0, 0.5}, {0, 0.5, 0.5}};
    q.clear();
    for (int i = 0; i < ncell; ++i)
        for (int j = 0; j < ncell; ++j)
            for (int k = 0; k < ncell; ++k)
                for (const auto& b : basis) {
                    q.push_back((i + b[0]) * a);
                    q.push_back((j + b[1]) * a);
                    q.push_back((k + b[2]) * a);
                }
    const size_t n = q.size() / 3;
    v.assign(q.size(), 0.0);
    double m[3] = {0, 0, 0};
    for (size_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            v[3 * i + d] = std::sin(0.37 * (double)i + 1.3 * d);
            m[d] += v[3 * i + d];
        }
    for (size_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) v[3 * i + d] -= m[d] / (double)n;
}

template <class T>
T* dev(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T) + 16) != hipSuccess) {
        std::fprintf(stderr, "host_check: hipMalloc failed\n");
        std::exit(2);
    }
    return static_cast<T*>(p);
}

void gpu_checks() {
    std::vector<double> q, v;
    fcc(10, 2.0, q, v);  // 4000 particles, density 0.5
    const int64_t n = (int64_t)q.size() / 3;
    double* dq = dev<double>(q.size());
    double* dv = dev<double>(v.size());
    double* dF = dev<double>(q.size());
    int32_t* dcell = dev<int32_t>(n);
    int64_t* dkp = dev<int64_t>(n + 1);
    (void)hipMemcpy(dq, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice);
    (void)hipMemcpy(dv, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
    const char* cache = "host_check_tune.txt";
    std::remove(cache);
    for (int prec : {MD_PREC_FP64, MD_PREC_FP32_MIXED}) {
        md_params p = base(n, 20.0);
        p.precision = prec;
        md_ctx* c = nullptr;
        OK(md_create(&p, nullptr, &c));
        if (!c) continue;
        CHECK(md_step(c, 1, 0) == MD_ESTATE);  // no state yet
        OK(md_set_state(c, dq, dv));
        OK(md_build_cells(c));
        int32_t nc[3] = {0, 0, 0};
        OK(md_get_cells(c, dcell, nc));
        CHECK(nc[0] == 7 && nc[1] == 7 && nc[2] == 7);
        OK(md_build_neighbors(c));
        int64_t total = -1;
        CHECK(md_get_neighbors(c, dkp, nullptr, 0, &total) == MD_EINVAL);  // count only: cap 0 < total
        CHECK(total > 0);
        int32_t* dpl = dev<int32_t>((size_t)total);
        CHECK(md_get_neighbors(c, dkp, dpl, total - 1, &total) == MD_EINVAL);
        OK(md_get_neighbors(c, dkp, dpl, total, &total));
        OK(md_compute_forces(c, dF));
        OK(md_set_timing(c, 1));
        OK(md_step(c, 30, 10));
        OK(md_set_timing(c, 0));
        double ke = 0.0, pe = 0.0, P = 0.0;
        OK(md_energy(c, &ke, &pe));
        CHECK(std::isfinite(ke) && std::isfinite(pe) && ke > 0.0);
        double kes[8], pes[8], vir[8], th[8];
        int32_t cnt = 0;
        OK(md_energy_series(c, kes, pes, 8, &cnt));
        CHECK(cnt == 3);
        OK(md_observable_series(c, vir, th, 8, &cnt));
        OK(md_pressure(c, &P));
        const double T = 1.0;
        OK(md_set_thermostat(c, &T, 0.5));
        OK(md_step(c, 10, 5));
        double xi = 0.0, eta = 0.0;
        OK(md_get_thermostat(c, &xi, &eta));
        OK(md_set_thermostat(c, nullptr, 0.0));
        OK(md_autotune(c, cache));  // timed, appended to the cache
        OK(md_autotune(c, cache));  // read back from the cache
        md_stats st;
        OK(md_get_stats(c, &st));
        CHECK(st.steps == 40 && st.ncell[0] >= 3 && st.cell_scale >= 1.0);
        const double s = 0.9;
        OK(md_scale_velocities(c, &s));
        OK(md_rescale_box(c, 1.1));
        CHECK(md_rescale_box(c, 0.1) == MD_EINVAL);
        OK(md_step(c, 5, 0));
        md_bubble_info bi, bj;
        int64_t roots[16], sizes[16], roots2[16], sizes2[16];
        OK(md_bubbles(c, 0, 3.0, 0.2, nullptr, nullptr, roots, sizes, 16, &bi));
        OK(md_bubbles_noalloc(c, 0, 3.0, 0.2, nullptr, nullptr, roots2, sizes2, 16, &bj));
        CHECK(bi.nbubbles == bj.nbubbles && bi.ngas == bj.ngas && bi.largest == bj.largest);
        CHECK(md_bubbles(c, 1, 3.0, 0.2, nullptr, nullptr, nullptr, nullptr, 0, &bi) == MD_EINVAL);
        CHECK(md_bubbles(c, 0, -1.0, 0.2, nullptr, nullptr, nullptr, nullptr, 0, &bi) == MD_EINVAL);
        CHECK(std::strlen(md_last_error(c)) > 0);
        OK(md_get_state(c, dq, dv));
        (void)hipFree(dpl);
        OK(md_destroy(c));
        (void)hipMemcpy(dq, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice);
        (void)hipMemcpy(dv, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
    }
    std::remove(cache);
    // ensemble of 3 boxes (the same lattice three times, boxes differ in nothing but
    // their place in the arrays), stepped in captured graphs
    {
        std::vector<double> q3, v3;
        for (int r = 0; r < 3; ++r) {
            q3.insert(q3.end(), q.begin(), q.end());
            v3.insert(v3.end(), v.begin(), v.end());
        }
        double* dq3 = dev<double>(q3.size());
        double* dv3 = dev<double>(v3.size());
        (void)hipMemcpy(dq3, q3.data(), q3.size() * sizeof(double), hipMemcpyHostToDevice);
        (void)hipMemcpy(dv3, v3.data(), v3.size() * sizeof(double), hipMemcpyHostToDevice);
        md_params b3[3] = {base(n, 20.0), base(n, 20.0), base(n, 20.0)};
        for (auto& p : b3) {
            p.precision = MD_PREC_FP32_MIXED;
            p.flags = MD_F_GRAPH;
        }
        hipStream_t stream;
        (void)hipStreamCreate(&stream);
        md_ctx* c = nullptr;
        OK(md_batch_create(b3, 3, stream, &c));
        if (c) {
            OK(md_set_state(c, dq3, dv3));
            OK(md_step(c, 40, 20));
            double ke[3], pe[3];
            OK(md_batch_energy(c, ke, pe));
            CHECK(ke[0] == ke[1] && ke[1] == ke[2] && pe[0] == pe[1] && pe[1] == pe[2]);
            OK(md_destroy(c));
        }
        // the same ensemble with a small list capacity and one box three times as
        // fast: its lists outgrow the capacity during stepping, the step stops at
        // that build, and the other boxes' lists move to the larger layout
        for (size_t i = 0; i < v.size(); ++i) v3[i] *= 3.0;
        (void)hipMemcpy(dv3, v3.data(), v3.size() * sizeof(double), hipMemcpyHostToDevice);
        for (auto& p : b3) {
            p.precision = MD_PREC_FP64;
            p.flags = 0;
            p.list_cap = 48;
            p.threads_per_key = 1;
        }
        c = nullptr;
        OK(md_batch_create(b3, 3, stream, &c));
        if (c) {
            OK(md_set_state(c, dq3, dv3));
            OK(md_step(c, 60, 20));
            md_stats st;
            OK(md_get_stats(c, &st));
            CHECK(st.list_regrows >= 1 && st.list_cap > 48 && st.steps == 60);
            double ke[3], pe[3];
            OK(md_batch_energy(c, ke, pe));
            CHECK(std::isfinite(ke[0]) && std::isfinite(pe[0]) && pe[1] == pe[2]);
            OK(md_destroy(c));
        }
        (void)hipStreamDestroy(stream);
        (void)hipFree(dq3);
        (void)hipFree(dv3);
    }
    (void)hipFree(dq);
    (void)hipFree(dv);
    (void)hipFree(dF);
    (void)hipFree(dcell);
    (void)hipFree(dkp);
}

}  // namespace

int main() {
    host_only_checks();
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        std::printf("host_check: no GPU; host-only checks: %s\n", g_fail ? "FAILED" : "passed");
        return g_fail ? 1 : 0;
    }
    gpu_checks();
    std::printf("host_check: host-only and GPU checks: %s (%d failures)\n", g_fail ? "FAILED" : "passed", g_fail);
    return g_fail ? 1 : 0;
}
