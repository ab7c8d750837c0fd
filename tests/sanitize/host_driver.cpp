// Sanitizer driver for the host runtimes (ch_host.cpp, dp_host.cpp built
// host-only with AddressSanitizer and UndefinedBehaviorSanitizer): every
// argument-validation path of the two C ABIs that returns before any device
// work, and the host-side line-solve coefficients.  Exit 0 when every call
// returns the expected status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/ch.h"
#include "../../include/dp.h"

static int failures = 0;
static void expect(bool ok, const char* what)
{
    if (!ok) {
        std::printf("FAILED: %s (%s)\n", what, ch_last_error(nullptr));
        ++failures;
    }
}

static ch_member_desc desc(int nx, int ny, int nz = 1)
{
    ch_member_desc d{};
    d.dim = nz > 1 ? 3 : 2;
    d.n[0] = nx;
    d.n[1] = ny;
    d.n[2] = nz;
    d.L[0] = d.L[1] = d.L[2] = 6.283185307179586;
    d.gamma = 0.01;
    d.dt = 1e-3;
    d.noise = 0.05;
    d.seed = 3;
    return d;
}

int main()
{
    // workspace sizes: valid ensembles of every kind, and refused shapes
    std::vector<ch_member_desc> ens = {desc(512, 512), desc(256, 256), desc(32, 16, 8), desc(40, 24)};
    for (int i = 0; i < 16; ++i) ens.push_back(desc(64, 32));
    expect(ch_workspace_bytes(ens.data(), (int32_t)ens.size(), CH_F32_BULK, 10, 101) > 0, "valid workspace");
    expect(ch_workspace_bytes(ens.data(), (int32_t)ens.size(), CH_F64, 1, 1) > 0, "valid workspace f64");
    const int bad_n[][3] = {{7, 64, 1}, {64, 4100, 1}, {66, 64, 1}, {260, 64, 1}, {8, 8, 0}};
    for (auto& b : bad_n) {
        ch_member_desc d = desc(b[0], b[1], b[2] > 0 ? b[2] : 1);
        if (b[2] == 0) d.n[2] = 0;
        expect(ch_workspace_bytes(&d, 1, CH_F64, 10, 2) == 0, "refused shape");
    }
    ch_member_desc g = desc(64, 64);
    g.gamma = -1.0;
    expect(ch_workspace_bytes(&g, 1, CH_F64, 10, 2) == 0, "refused gamma");
    g = desc(64, 64);
    g.dt = NAN;
    expect(ch_workspace_bytes(&g, 1, CH_F64, 10, 2) == 0, "refused dt");
    expect(ch_workspace_bytes(nullptr, 1, CH_F64, 10, 2) == 0, "NULL members");
    expect(ch_workspace_bytes(ens.data(), 0, CH_F64, 10, 2) == 0, "no members");
    expect(ch_workspace_bytes(ens.data(), 1, (ch_precision)7, 10, 2) == 0, "bad precision");
    expect(ch_workspace_bytes(ens.data(), 1, CH_F64, 0, 2) == 0, "bad cadence");

    // ch_create: refused before any device call
    ch_ctx* ctx = nullptr;
    alignas(256) static unsigned char fake[1024];
    expect(ch_create(ens.data(), 1, CH_F64, CH_ENERGY_QUARTER, 10, 2, fake, sizeof fake, nullptr, nullptr) == CH_EINVAL,
           "NULL out");
    expect(ch_create(ens.data(), 1, CH_F64, CH_ENERGY_QUARTER, 10, 2, nullptr, 0, nullptr, &ctx) == CH_EINVAL,
           "NULL workspace");
    expect(ch_create(ens.data(), 1, CH_F64, CH_ENERGY_QUARTER, 10, 2, fake + 8, 512, nullptr, &ctx) == CH_EINVAL,
           "misaligned workspace");
    expect(ch_create(ens.data(), 1, CH_F64, (ch_energy_conv)5, 10, 2, fake, sizeof fake, nullptr, &ctx) == CH_EINVAL,
           "bad convention");
    expect(ch_create(ens.data(), 1, CH_F64, CH_ENERGY_QUARTER, 10, 2, fake, sizeof fake, nullptr, &ctx) == CH_ENOMEM,
           "workspace too small");
    expect(ctx == nullptr, "no context on failure");

    // every context call on a pointer that is not a live context
    ch_ctx* bogus = reinterpret_cast<ch_ctx*>(fake);
    double d1 = 0, d2 = 0;
    int64_t n = 0;
    int32_t nc = 0;
    char buf[64];
    expect(ch_init_random(bogus) == CH_ESTATE, "init on unknown ctx");
    expect(ch_step(bogus, 1) == CH_ESTATE, "step on unknown ctx");
    expect(ch_energy(bogus, &d1, &d2) == CH_ESTATE, "energy on unknown ctx");
    expect(ch_get_step(bogus, &n) == CH_ESTATE, "get_step on unknown ctx");
    expect(ch_set_theta(bogus, 0.5) == CH_ESTATE, "set_theta on unknown ctx");
    expect(ch_num_classes(bogus, &nc) == CH_ESTATE, "num_classes on unknown ctx");
    expect(ch_describe(bogus, buf, sizeof buf) == CH_ESTATE, "describe on unknown ctx");
    expect(ch_destroy(bogus) == CH_ESTATE, "destroy unknown ctx");
    expect(ch_step(nullptr, 1) == CH_EINVAL, "step on NULL");
    expect(std::strlen(ch_last_error(nullptr)) > 0, "error message");

    // allocation-free stepping: argument checks before anything is enqueued
    double* field = reinterpret_cast<double*>(fake);
    std::vector<ch_member_desc> big(32, desc(1024, 1024));
    expect(ch_step_static(big.data(), 32, CH_F32_BULK, field, 1, nullptr, nullptr) == CH_ENOMEM, "static oversize");
    expect(ch_step_static(ens.data(), 0, CH_F64, field, 1, nullptr, nullptr) == CH_EINVAL, "static m = 0");
    expect(ch_step_static(ens.data(), 2, CH_F64, field, 1, nullptr, nullptr) == CH_EINVAL, "static mixed grids");
    expect(ch_step_static(ens.data(), 1, CH_F64, nullptr, 1, nullptr, nullptr) == CH_EINVAL, "static NULL field");
    expect(ch_step_static(ens.data(), 1, CH_F64, fake + 4, 1, nullptr, nullptr) == CH_EINVAL, "static misaligned");
    expect(ch_step_static(ens.data(), 1, CH_F64, field, -1, nullptr, nullptr) == CH_EINVAL, "static nsteps");

    // host-side line-solve coefficients: the DC gain of the factorisation is 1
    double co[11];
    const double rhos[] = {1e-4, 1.72, 441.0, 1764.0, 1e6};
    for (double rho : rhos)
        for (int chunk : {4, 16, 64}) {
            expect(ch_solver_coefficients(rho, 512, chunk, 0, co) == CH_OK, "coefficients");
            const double q = 1.0 - co[0] - co[1];
            expect(std::fabs(co[2] * (1.0 / (q * q)) - 1.0) < 1e-12, "DC gain");
        }
    expect(ch_solver_coefficients(-1.0, 512, 16, 0, co) == CH_EINVAL, "coefficients rho");

    // droplet ensembles
    dp_params prm{};
    prm.t_end = 1.0;
    prm.dt_sample = 0.1;
    prm.rtol = 1e-6;
    prm.atol = 1e-9;
    prm.h0 = 1e-4;
    prm.max_attempts = 1000;
    const int32_t sizes[] = {128, 8192, 1};
    expect(dp_workspace_bytes(sizes, 3, &prm) > 0, "dp workspace");
    const int32_t too_big[] = {8193};
    expect(dp_workspace_bytes(too_big, 1, &prm) == 0, "dp too many droplets");
    dp_params bad = prm;
    bad.rtol = 0.0;
    expect(dp_workspace_bytes(sizes, 3, &bad) == 0, "dp rtol");
    dp_ctx* dctx = nullptr;
    expect(dp_create(sizes, 3, &prm, nullptr, 0, nullptr, &dctx) == CH_EINVAL, "dp NULL workspace");
    expect(dp_create(sizes, 3, &prm, fake, sizeof fake, nullptr, &dctx) == CH_EINVAL, "dp workspace too small");
    dp_ctx* dbogus = reinterpret_cast<dp_ctx*>(fake);
    expect(dp_advance(dbogus, 1) == CH_ESTATE, "dp advance on unknown ctx");
    expect(dp_destroy(dbogus) == CH_ESTATE, "dp destroy unknown ctx");

    std::printf(failures ? "host driver: %d FAILED\n" : "host driver: ok\n", failures);
    return failures ? 1 : 0;
}
