// AddressSanitizer / UndefinedBehaviorSanitizer run of the library's host
// code (test infrastructure): descriptor validation and workspace layout,
// the relaxation-map labelling, map checks of fw2_create_domain on exact-size
// host maps and its clean-up when the device calls fail, and the argument
// checks of every entry point, all without a GPU (the device launchers are
// replaced by tests/sanitize/launch_stubs.cpp).  Exit status 0 when every
// check held.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fw2.h"

static int g_fail = 0;
#define CHECK(cond)                                                  \
    do {                                                             \
        if (!(cond)) {                                               \
            std::printf("check failed line %d: %s\n", __LINE__, #cond); \
            ++g_fail;                                                \
        }                                                            \
    } while (0)

struct Maps {
    std::vector<float> c, rho, beta;
    std::vector<uint8_t> label;
    std::vector<double> table;
};

static fw2_domain_desc desc_for(Maps &m, int ndim, int64_t nx, int64_t ny, int64_t nz, int L, int labels)
{
    fw2_domain_desc d;
    std::memset(&d, 0, sizeof(d));
    d.ndim = ndim;
    d.n_relax = L;
    d.n[0] = nx;
    d.n[1] = ny;
    d.n[2] = ndim == 3 ? nz : 1;
    d.h = 5e-5;
    d.dt = 0.3 * 5e-5 / 1600.0;
    for (int a = 0; a < ndim; ++a) {
        d.bound_cells[a] = 2;
        d.trans_cells[a] = 1;
    }
    d.pml_Rc = 1e-3;
    d.pml_npoly = 2;
    d.relax_scheme = FW2_RELAX_CENTRED;
    const size_t n = (size_t)nx * ny * (ndim == 3 ? nz : 1);
    m.c.assign(n, 1540.0f);
    m.rho.assign(n, 1000.0f);
    m.beta.assign(n, 3.5f);
    m.label.assign(n, 0);
    for (size_t i = 0; i < n; ++i) m.label[i] = (uint8_t)(i % labels);
    m.table.assign((size_t)labels * (2 + 4 * L), 0.0);
    for (int r = 0; r < labels; ++r) {
        m.table[(size_t)r * (2 + 4 * L)] = 1.0;
        m.table[(size_t)r * (2 + 4 * L) + 1] = 1.0;
        for (int q = 2; q < 2 + 4 * L; ++q) m.table[(size_t)r * (2 + 4 * L) + q] = 1e4 * (q + r);
    }
    d.c = m.c.data();
    d.rho = m.rho.data();
    d.beta = m.beta.data();
    d.label = labels > 1 ? m.label.data() : nullptr;
    d.n_labels = labels;
    d.relax_table = m.table.data();
    return d;
}

static void workspace_checks()
{
    Maps m;
    uint64_t b = 0;
    const int shapes[][4] = {{2, 1, 1, 1}, {2, 17, 5, 1}, {2, 300, 7, 1}, {3, 5, 6, 7}, {3, 33, 2, 9}};
    for (auto &s : shapes)
        for (int L = 1; L <= 8; ++L) {
            fw2_domain_desc d = desc_for(m, s[0], s[1], s[2], s[3], L, 3);
            for (int a = 0; a < s[0]; ++a)
                if (d.n[a] < 4) d.bound_cells[a] = d.trans_cells[a] = 0;
            CHECK(fw2_workspace_bytes(&d, &b) == FW2_OK);
            CHECK(b > (uint64_t)(1 + s[0] + 2 * s[0] * L) * (uint64_t)d.n[0] * 4);
        }
    fw2_domain_desc d = desc_for(m, 2, 40, 30, 1, 2, 2);
    fw2_domain_desc e = d;
    e.n[0] = 32768;
    e.n[1] = 32768;
    CHECK(fw2_workspace_bytes(&e, &b) == FW2_E_INVALID);
    e = d;
    e.ndim = 4;
    CHECK(fw2_workspace_bytes(&e, &b) == FW2_E_INVALID);
    e = d;
    e.nonlinear_form = 7;
    CHECK(fw2_workspace_bytes(&e, &b) == FW2_E_INVALID);
    e = d;
    e.slab_nz = 64;
    CHECK(fw2_workspace_bytes(&e, &b) == FW2_E_INVALID);
    e = d;
    e.map_kind = 5;
    CHECK(fw2_workspace_bytes(&e, &b) == FW2_E_INVALID);
    CHECK(fw2_workspace_bytes(nullptr, &b) == FW2_E_INVALID);
    CHECK(fw2_workspace_bytes(&d, nullptr) == FW2_E_INVALID);
    CHECK(std::strlen(fw2_last_error()) > 0);
}

static void label_map_checks()
{
    unsigned seed = 7;
    auto rnd = [&seed]() {
        seed = seed * 1103515245u + 12345u;
        return (seed >> 8) & 0xffffff;
    };
    for (int L = 1; L <= 8; ++L)
        for (int64_t n : {1, 2, 97, 4000}) {
            const int nrow = 2 + 4 * L;
            const int distinct = 1 + (int)(rnd() % 200);
            std::vector<double> rows((size_t)distinct * nrow);
            for (auto &x : rows) x = (double)(rnd() % 1000) + 0.5;
            std::vector<double> maps((size_t)nrow * n);
            std::vector<int> which(n);
            for (int64_t i = 0; i < n; ++i) {
                which[i] = (int)(rnd() % distinct);
                for (int q = 0; q < nrow; ++q) maps[(size_t)q * n + i] = rows[(size_t)which[i] * nrow + q];
            }
            std::vector<uint8_t> lab(n);
            std::vector<double> table((size_t)FW2_MAX_LABELS * nrow);
            int32_t nl = 0;
            CHECK(fw2_label_relaxation_map(n, L, maps.data(), lab.data(), table.data(), &nl) == FW2_OK);
            CHECK(nl >= 1 && nl <= distinct);
            for (int64_t i = 0; i < n; ++i)
                for (int q = 0; q < nrow; ++q)
                    CHECK(table[(size_t)lab[i] * nrow + q] == maps[(size_t)q * n + i]);
        }
    const int L = 2, nrow = 2 + 4 * L, n = 300;
    std::vector<double> maps((size_t)nrow * n);
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < nrow; ++q) maps[(size_t)q * n + i] = i + 0.25 * q;
    std::vector<uint8_t> lab(n);
    std::vector<double> table((size_t)FW2_MAX_LABELS * nrow);
    int32_t nl = 0;
    CHECK(fw2_label_relaxation_map(n, L, maps.data(), lab.data(), table.data(), &nl) == FW2_E_INVALID);
    CHECK(fw2_label_relaxation_map(n, 9, maps.data(), lab.data(), table.data(), &nl) == FW2_E_INVALID);
    CHECK(fw2_label_relaxation_map(0, L, maps.data(), lab.data(), table.data(), &nl) == FW2_E_INVALID);
    CHECK(fw2_label_relaxation_map(n, L, nullptr, lab.data(), table.data(), &nl) == FW2_E_INVALID);
}

static void create_checks()
{
    // The host maps are checked on exact-size arrays; without a device the
    // first runtime call fails and the half-built domain is released.
    const int shapes[][4] = {{2, 19, 11, 1}, {3, 7, 6, 5}};
    for (auto &s : shapes) {
        Maps m;
        fw2_domain_desc d = desc_for(m, s[0], s[1], s[2], s[3], 2, 3);
        uint64_t b = 0;
        CHECK(fw2_workspace_bytes(&d, &b) == FW2_OK);
        void *ws = std::aligned_alloc(256, (b + 255) / 256 * 256);
        fw2_domain *dom = nullptr;
        fw2_status st = fw2_create_domain(&d, ws, b, &dom);
        CHECK(st != FW2_OK && dom == nullptr);
        CHECK(fw2_create_domain(&d, ws, b - 1, &dom) == FW2_E_NOMEM);
        CHECK(fw2_create_domain(&d, (char *)ws + 8, b, &dom) == FW2_E_INVALID);
        m.c[m.c.size() - 1] = -1.0f;                // a bad last sample is found
        CHECK(fw2_create_domain(&d, ws, b, &dom) == FW2_E_INVALID);
        m.c[m.c.size() - 1] = 1540.0f;
        m.label[m.label.size() - 1] = 9;            // label >= n_labels
        CHECK(fw2_create_domain(&d, ws, b, &dom) == FW2_E_INVALID);
        std::free(ws);
    }
}

static void null_checks()
{
    uint64_t b = 0;
    double ms[2];
    int64_t cnt[2];
    CHECK(fw2_step(nullptr, 1) == FW2_E_STATE);
    CHECK(fw2_step_phase(nullptr, 0) == FW2_E_STATE);
    CHECK(fw2_step_into(nullptr, 1, nullptr, nullptr) == FW2_E_STATE);
    CHECK(fw2_halo_bytes(nullptr, FW2_HALO_P, &b) == FW2_E_STATE);
    CHECK(fw2_halo_pack(nullptr, FW2_HALO_P, FW2_LOW, nullptr) == FW2_E_STATE);
    CHECK(fw2_halo_unpack(nullptr, FW2_HALO_V, FW2_HIGH, nullptr) == FW2_E_STATE);
    CHECK(fw2_read_fields(nullptr, FW2_FIELD_P, nullptr, FW2_HOST) == FW2_E_STATE);
    CHECK(fw2_get_kernel_timing(nullptr, ms, cnt) == FW2_E_STATE);
    CHECK(fw2_adjoint_begin(nullptr, nullptr, 0) == FW2_E_STATE);
    CHECK(fw2_batch_step(nullptr, 1) == FW2_E_STATE);
    fw2_batch *bt = nullptr;
    CHECK(fw2_batch_create_noalloc(65, nullptr, &bt) == FW2_E_INVALID && bt == nullptr);
    CHECK(fw2_batch_create_noalloc(4, nullptr, &bt) != FW2_OK && bt == nullptr);
    CHECK(fw2_current_step(nullptr) == -1);
    alignas(256) static unsigned char probe_buf[512];
    CHECK(fw2_stream_probe(7, probe_buf, 1 << 20, nullptr) == FW2_E_INVALID);
    CHECK(fw2_stream_probe(FW2_PROBE_COPY, nullptr, 1 << 20, nullptr) == FW2_E_INVALID);
    CHECK(fw2_stream_probe(FW2_PROBE_COPY, probe_buf + 4, 1 << 20, nullptr) == FW2_E_INVALID);
    CHECK(fw2_stream_probe(FW2_PROBE_VELOCITY_MIX, probe_buf, 1024, nullptr) == FW2_E_INVALID);
    CHECK(fw2_stream_probe(FW2_PROBE_VELOCITY_MIX, probe_buf, ((uint64_t)1 << 40) + 1, nullptr) == FW2_E_INVALID);
    CHECK(fw2_stream_probe(FW2_PROBE_COPY, probe_buf, 1 << 20, nullptr) == FW2_E_HIP);   // the stub launcher: no device
    fw2_destroy_domain(nullptr);
    fw2_batch_destroy(nullptr);
}

int main()
{
    workspace_checks();
    label_map_checks();
    create_checks();
    null_checks();
    std::printf("library host sanitizer checks: %d failed\n", g_fail);
    return g_fail ? 1 : 0;
}
