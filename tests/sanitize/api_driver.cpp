// Drives libtri's C ABI built for the CPU against the stub runtime
// (api_stubs.cpp) under AddressSanitizer/UndefinedBehaviorSanitizer: argument
// and shape validation of every entry point (refusals launch nothing and leave
// the data untouched), the no-allocation / no-synchronisation promise of the
// solves, workspace refusal and tri_reserve, plans with ragged items, capture
// and destruction.  Exit status 0 when every check holds.
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tri.h"

extern int g_launches, g_mallocs, g_frees, g_syncs, g_symbol_lookups;

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #cond);         \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

// A refused call: the expected status, nothing launched or allocated, data kept.
#define REFUSED(call, want, buf)                                                 \
    do {                                                                         \
        const std::vector<double> before_ = (buf);                               \
        const int l0_ = g_launches, m0_ = g_mallocs;                             \
        const tri_status st_ = (call);                                           \
        if (st_ != (want))                                                       \
            std::fprintf(stderr, "line %d: status %d, want %d\n", __LINE__, (int)st_, (int)(want)); \
        CHECK(st_ == (want));                                                    \
        CHECK(g_launches == l0_ && g_mallocs == m0_);                            \
        CHECK(before_ == (buf));                                                 \
    } while (0)

int main()
{
    tri_ctx ctx = nullptr;
    CHECK(tri_create(nullptr, 0, nullptr) == TRI_E_ARG);
    CHECK(tri_create(&ctx, 3, nullptr) == TRI_E_ARG);
    CHECK(tri_create(&ctx, 0, nullptr) == TRI_OK && ctx);

    const int64_t Nx = 64, Ny = 32, Nz = 24;
    std::vector<double> u(Nx * Ny * Nz, 1.0), ax(Nx, -0.1), bx(Nx, 1.2), cx(Nx, -0.1);
    std::vector<double> ay(Ny, -0.1), by(Ny, 1.2), cy(Ny, -0.1), az(Nz, -0.1), bz(Nz, 1.2), cz(Nz, -0.1);

    // ---- null context on every entry point --------------------------------
    tri_coef C{ax.data(), bx.data(), cx.data(), 1, 0, 0};
    tri_lines L{Nx, Ny * Nz, 1, 1, Nx, 0};
    CHECK(tri_pdd_solve(nullptr, &C, &L, TRI_REAL, u.data(), 4, 0, TRI_F64, nullptr) == TRI_E_ARG);
    CHECK(tri_ppt_solve(nullptr, &C, &L, TRI_REAL, u.data(), 4, 0, TRI_F64, nullptr) == TRI_E_ARG);
    CHECK(adi_sweep(nullptr, 0, u.data(), Nx, Ny, Nz, ax.data(), bx.data(), cx.data(), 4, 0, 0, TRI_F64,
                    nullptr) == TRI_E_ARG);
    CHECK(tri_reserve(nullptr, 64, 4, 1) == TRI_E_ARG);
    CHECK(tri_sync_status(nullptr) == TRI_E_ARG);
    CHECK(tri_set_pdd_tolerance(nullptr, 1.0) == TRI_E_ARG);
    CHECK(tri_plan_execute(nullptr) == TRI_E_ARG);
    CHECK(tri_plan_destroy(nullptr) == TRI_E_ARG);
    CHECK(tri_stream_copy(nullptr, u.data(), u.data(), 4) == TRI_E_ARG);

    // ---- shape and argument refusals --------------------------------------
    REFUSED(tri_pdd_solve(ctx, &C, &L, TRI_REAL, u.data(), 5, 0, TRI_F64, nullptr), TRI_E_SHAPE, u);  // 64 % 5
    REFUSED(tri_pdd_solve(ctx, &C, &L, TRI_REAL, u.data(), 0, 0, TRI_F64, nullptr), TRI_E_SHAPE, u);
    REFUSED(tri_pdd_solve(ctx, &C, &L, TRI_REAL, u.data(), 32, 0, TRI_F64, nullptr), TRI_E_SHAPE, u);  // > 16
    REFUSED(tri_pdd_solve(ctx, &C, &L, TRI_REAL, u.data(), 4, 2, TRI_F64, nullptr), TRI_E_ARG, u);    // periodic 2
    REFUSED(tri_pdd_solve(ctx, &C, &L, (tri_field)5, u.data(), 4, 0, TRI_F64, nullptr), TRI_E_ARG, u);
    REFUSED(tri_pdd_solve(ctx, &C, &L, TRI_REAL, u.data(), 4, 0, (tri_prec)7, nullptr), TRI_E_ARG, u);
    REFUSED(tri_pdd_solve(ctx, &C, &L, TRI_REAL, nullptr, 4, 0, TRI_F64, nullptr), TRI_E_ARG, u);
    REFUSED(tri_pdd_solve(ctx, nullptr, &L, TRI_REAL, u.data(), 4, 0, TRI_F64, nullptr), TRI_E_ARG, u);
    {
        tri_lines bad = L;
        bad.nb0 = -1;
        REFUSED(tri_pdd_solve(ctx, &C, &bad, TRI_REAL, u.data(), 4, 0, TRI_F64, nullptr), TRI_E_ARG, u);
        tri_lines empty = L;
        empty.nb0 = 0;
        REFUSED(tri_pdd_solve(ctx, &C, &empty, TRI_REAL, u.data(), 4, 0, TRI_F64, nullptr), TRI_OK, u);
        tri_lines two = {2, 8, 1, 1, 2, 0};
        REFUSED(tri_ppt_solve(ctx, &C, &two, TRI_REAL, u.data(), 1, 1, TRI_F64, nullptr), TRI_E_SHAPE, u);  // periodic n < 3
    }
    REFUSED(adi_sweep(ctx, 3, u.data(), Nx, Ny, Nz, ax.data(), bx.data(), cx.data(), 4, 0, 0, TRI_F64, nullptr),
            TRI_E_ARG, u);
    REFUSED(adi_sweep(ctx, 0, u.data(), -1, Ny, Nz, ax.data(), bx.data(), cx.data(), 4, 0, 0, TRI_F64, nullptr),
            TRI_E_ARG, u);
    REFUSED(adi_sweep(ctx, 0, u.data(), Nx, Ny, Nz, ax.data(), bx.data(), cx.data(), 4, 0, 9, TRI_F64, nullptr),
            TRI_E_ARG, u);
    REFUSED(tri_set_pdd_tolerance(ctx, std::nan("")), TRI_E_ARG, u);
    REFUSED(tri_stream_copy(ctx, u.data() + 1, u.data(), 8), TRI_E_ARG, u);   // partial overlap / misaligned
    REFUSED(tri_stream_copy(ctx, u.data(), u.data(), -1), TRI_E_ARG, u);

    // ---- a solve launches, but never allocates or synchronises -------------
    {
        const int l0 = g_launches, m0 = g_mallocs, f0 = g_frees, s0 = g_syncs;
        CHECK(adi_sweep(ctx, 0, u.data(), Nx, Ny, Nz, ax.data(), bx.data(), cx.data(), 8, 0, 0, TRI_F64, nullptr) ==
              TRI_OK);
        CHECK(adi_sweep(ctx, 1, u.data(), Nx, Ny, Nz, ay.data(), by.data(), cy.data(), 4, 0, 0, TRI_F64, nullptr) ==
              TRI_OK);
        CHECK(adi_sweep(ctx, 2, u.data(), Nx, Ny, Nz, az.data(), bz.data(), cz.data(), 4, 1, 1, TRI_F32_REFINE,
                        nullptr) == TRI_OK);
        CHECK(g_launches > l0);
        CHECK(g_mallocs == m0 && g_frees == f0 && g_syncs == s0);
    }

    // ---- the allocation-free sweep: static scratch, looked up once per device
    {
        CHECK(g_symbol_lookups == 1);
        tri_ctx ctx2 = nullptr;
        CHECK(tri_create(&ctx2, 0, nullptr) == TRI_OK);
        CHECK(g_symbol_lookups == 1);                      // already bound for device 0
        CHECK(tri_destroy(ctx2) == TRI_OK);
        const int l0 = g_launches, m0 = g_mallocs, f0 = g_frees, s0 = g_syncs;
        for (int d = 0; d < 3; ++d) {
            const double *A = d == 0 ? ax.data() : (d == 1 ? ay.data() : az.data());
            const double *B = d == 0 ? bx.data() : (d == 1 ? by.data() : bz.data());
            const double *Cc = d == 0 ? cx.data() : (d == 1 ? cy.data() : cz.data());
            CHECK(adi_sweep_noalloc(ctx, d, u.data(), Nx, Ny, Nz, A, B, Cc, 4, d == 2, TRI_PDD, TRI_F64) == TRI_OK);
        }
        CHECK(g_launches > l0 && g_mallocs == m0 && g_frees == f0 && g_syncs == s0);
        // 16384 rows: about 1.4 MB of tables, beyond the 1 MiB scratch
        std::vector<double> big(16384, 1.0), ab(16384, -0.1), bb(16384, 1.2), cb(16384, -0.1);
        REFUSED(adi_sweep_noalloc(ctx, 0, big.data(), 16384, 1, 1, ab.data(), bb.data(), cb.data(), 8, 0, TRI_PDD,
                                  TRI_F64), TRI_E_NOMEM, big);
        REFUSED(adi_sweep_noalloc(nullptr, 0, big.data(), 16384, 1, 1, ab.data(), bb.data(), cb.data(), 8, 0,
                                  TRI_PDD, TRI_F64), TRI_E_ARG, big);
        REFUSED(adi_sweep_noalloc(ctx, 0, big.data(), 16384, 1, 1, ab.data(), bb.data(), cb.data(), 3, 0, TRI_PDD,
                                  TRI_F64), TRI_E_SHAPE, big);
    }

    // ---- workspace: a call whose tables do not fit is refused, tri_reserve grows it
    {
        const int64_t Nk = 200000;   // 200000 matrices of 32 rows: beyond the 64 MiB workspace
        std::vector<double> ph(2 * 4 * Ny, 0.5), lam(Nk, 1.0);
        REFUSED(poisson_wavenumber_solve(ctx, ph.data(), 4, Ny, Nk, ay.data(), cy.data(), lam.data(), 4, TRI_F64, 2,
                                         nullptr), TRI_E_NOMEM, ph);
        CHECK(tri_reserve(ctx, Ny, 4, Nk) == TRI_OK);
        CHECK(tri_reserve(ctx, 0, 4, 1) == TRI_E_ARG);
        CHECK(tri_reserve(ctx, 64, 17, 1) == TRI_E_ARG);
    }

    // ---- per-line pivot record: shared matrices refused, null piv refused --
    {
        std::vector<unsigned char> piv(Nx * Ny * Nz);
        tri_lines Ly{Ny, Nx, Nz, Nx, 1, Nx * Ny};
        tri_coef shared{ay.data(), by.data(), cy.data(), 1, 0, 0};
        REFUSED(tri_ppt_pivots(ctx, &shared, &Ly, u.data(), 4, 0, piv.data()), TRI_E_UNSUPPORTED, u);
        std::vector<double> A(Ny * Nx * Nz, -0.1), B(Ny * Nx * Nz, 1.2), Cc(Ny * Nx * Nz, -0.1);
        tri_coef per_line{A.data(), B.data(), Cc.data(), Nx, 1, Nx * Ny};
        REFUSED(tri_ppt_pivots(ctx, &per_line, &Ly, u.data(), 4, 0, nullptr), TRI_E_ARG, u);
        CHECK(tri_ppt_pivots(ctx, &per_line, &Ly, u.data(), 4, 0, piv.data()) == TRI_OK);
    }

    // ---- pressure steps: overlap, alignment, shape -----------------------
    {
        const int64_t nk = Nz / 2 + 1;
        std::vector<double> v(Nz * (Ny + 1) * Nx, 0.0), w(Nz * Ny * Nx, 0.0), uf(Nz * Ny * (Nx + 1), 0.0);
        std::vector<double> dy(Ny, 1.0 / Ny), phi(Nz * Ny * Nx), ph(2 * nk * Ny * Nx), lz(nk, 1.0), lx(Nx, 1.0);
        REFUSED(projection3d_step(ctx, uf.data(), v.data(), w.data(), 1.0 / Nx, dy.data(), 1.0 / Nz, ay.data(),
                                  cy.data(), lz.data(), lx.data(), ph.data(), v.data(), Nx, Ny, Nz, 4),
                TRI_E_ARG, v);                                             // phi overlaps v
        REFUSED(projection3d_step(ctx, uf.data(), v.data(), w.data(), 1.0 / Nx, dy.data(), 1.0 / Nz, ay.data(),
                                  cy.data(), lz.data(), lx.data(), ph.data() + 1, phi.data(), Nx, Ny, Nz, 4),
                TRI_E_ARG, v);                                             // spectrum not 16-byte aligned
        REFUSED(projection3d_step(ctx, uf.data(), v.data(), w.data(), 1.0 / Nx, dy.data(), 1.0 / Nz, ay.data(),
                                  cy.data(), lz.data(), lx.data(), ph.data(), phi.data(), Nx, Ny, 23, 4),
                TRI_E_SHAPE, v);                                           // odd Nz
        REFUSED(projection3d_step(ctx, uf.data(), v.data(), w.data(), 1.0 / Nx, dy.data(), 1.0 / Nz, ay.data(),
                                  cy.data(), lz.data(), lx.data(), ph.data(), phi.data(), Nx, Ny, Nz, 3),
                TRI_E_SHAPE, v);                                           // 32 % 3
        REFUSED(spanwise_rfft(ctx, w.data(), ph.data(), Ny * Nx, 14), TRI_E_UNSUPPORTED, w);   // Nz/2 = 7
        const int l0 = g_launches, m0 = g_mallocs, s0 = g_syncs;
        CHECK(projection3d_step(ctx, uf.data(), v.data(), w.data(), 1.0 / Nx, dy.data(), 1.0 / Nz, ay.data(),
                                cy.data(), lz.data(), lx.data(), ph.data(), phi.data(), Nx, Ny, Nz, 4) == TRI_OK);
        CHECK(g_launches > l0 && g_mallocs == m0 && g_syncs == s0);
        REFUSED(streamwise_dct(ctx, ph.data(), 14, 2), TRI_E_UNSUPPORTED, ph);   // 14 = 2 * 7
        REFUSED(streamwise_dct(ctx, ph.data(), 7, 2), TRI_E_SHAPE, ph);
    }

    // ---- plans: ragged items, execute without allocating, capture ---------
    {
        std::vector<double> u2(128 * 16 * 12, 1.0), a2(128, -0.1), b2(128, 1.2), c2(128, -0.1);
        std::vector<double> a16(16, -0.1), b16(16, 1.2), c16(16, -0.1), a12(12, -0.1), b12(12, 1.2), c12(12, -0.1);
        std::vector<double> ph2(2 * 7 * 16 * 128), lam2(7, 1.0), my(16, 1.0), mc(16, 1.0);
        lam2[0] = 0.0;
        my[0] = 0.0;
        mc[15] = 0.0;
        tri_item items[] = {
            {TRI_ITEM_ADI_X, u.data(), Nx, Ny, Nz, ax.data(), bx.data(), cx.data(), nullptr, 0, 0, TRI_PDD},
            {TRI_ITEM_ADI_Y, u.data(), Nx, Ny, Nz, ay.data(), by.data(), cy.data(), nullptr, 4, 0, TRI_PDD},
            {TRI_ITEM_ADI_Z, u.data(), Nx, Ny, Nz, az.data(), bz.data(), cz.data(), nullptr, 0, 1, TRI_PDD},
            {TRI_ITEM_ADI_X, u2.data(), 128, 16, 12, a2.data(), b2.data(), c2.data(), nullptr, 8, 0, TRI_PDD},
            {TRI_ITEM_ADI_Y, u2.data(), 128, 16, 12, a16.data(), b16.data(), c16.data(), nullptr, 2, 0, TRI_PPT},
            {TRI_ITEM_ADI_Z, u2.data(), 128, 16, 12, a12.data(), b12.data(), c12.data(), nullptr, 2, 1, TRI_PDD},
            {TRI_ITEM_POISSON, ph2.data(), 128, 16, 7, my.data(), nullptr, mc.data(), lam2.data(), 4, 0, TRI_PPT},
        };
        // every grouping of a level's launches (one launch per solve, per kernel
        // instance, per level): execute queues exactly the launches it reports
        for (const char *batch : {"0", "1", "2"}) {
            setenv("TRI_BATCH", batch, 1);
            tri_plan plan = nullptr;
            CHECK(tri_plan_create(ctx, items, 7, TRI_F64, &plan) == TRI_OK && plan);
            if (!plan) continue;
            const int n = tri_plan_launch_count(plan), l0 = g_launches;
            CHECK(n >= 1 && n <= 7);
            CHECK(tri_plan_execute(plan) == TRI_OK);
            CHECK(g_launches - l0 == n);
            CHECK(tri_plan_destroy(plan) == TRI_OK);
        }
        unsetenv("TRI_BATCH");
        CHECK(tri_plan_launch_count(nullptr) == -1);
        for (tri_prec prec : {TRI_F64, TRI_F32_REFINE}) {
            tri_plan plan = nullptr;
            CHECK(tri_plan_create(ctx, items, 7, prec, &plan) == TRI_OK && plan);
            if (!plan) continue;
            for (int i = 0; i < 7; ++i) CHECK(tri_plan_item_partitions(plan, i) >= 1);
            CHECK(tri_plan_item_partitions(plan, 7) == -1);
            char buf[256];
            CHECK(tri_plan_item_describe(plan, 0, buf, sizeof buf) > 0);
            CHECK(tri_plan_item_describe(plan, 9, buf, sizeof buf) == -1);
            const int l0 = g_launches, m0 = g_mallocs, s0 = g_syncs;
            CHECK(tri_plan_execute(plan) == TRI_OK);
            CHECK(g_launches > l0 && g_mallocs == m0 && g_syncs == s0);
            void *exec = nullptr;
            CHECK(tri_plan_capture(plan, &exec) == TRI_OK && exec);
            CHECK(tri_plan_graph_launch(plan) == TRI_OK);
            CHECK(tri_plan_destroy(plan) == TRI_OK);
        }
        tri_item bad = items[1];
        bad.P = 5;
        tri_plan plan = nullptr;
        const int m0 = g_mallocs;
        CHECK(tri_plan_create(ctx, &bad, 1, TRI_F64, &plan) == TRI_E_SHAPE && !plan);
        CHECK(g_mallocs == m0);
        bad = items[0];
        bad.kind = 9;
        CHECK(tri_plan_create(ctx, &bad, 1, TRI_F64, &plan) == TRI_E_ARG && !plan);
    }

    // ---- the fractional-step time step: set-up validation, steps allocate nothing
    {
        const int64_t nx = 16, ny = 32, nz = 24;
        std::vector<double> dyv(ny, 1.0 / ny);
        tri_ns_config cfg{nx, ny, nz, 1.0 / nx, 1.0 / nz, dyv.data(), 1e-3, 1e-3, {2, 4, 4}, 4};
        tri_ns ns = nullptr;
        const int m0 = g_mallocs;
        tri_ns_config bad = cfg;
        bad.Nx = 15;
        CHECK(ns_create(ctx, &bad, &ns) == TRI_E_SHAPE && !ns);
        bad = cfg;
        bad.Nz = 22;                                      // Nz/2 = 11
        CHECK(ns_create(ctx, &bad, &ns) == TRI_E_UNSUPPORTED && !ns);
        bad = cfg;
        bad.P_poisson = 3;
        CHECK(ns_create(ctx, &bad, &ns) == TRI_E_SHAPE && !ns);
        bad = cfg;
        bad.dt = 0.0;
        CHECK(ns_create(ctx, &bad, &ns) == TRI_E_ARG && !ns);
        bad = cfg;
        bad.dy = nullptr;
        CHECK(ns_create(ctx, &bad, &ns) == TRI_E_ARG && !ns);
        CHECK(g_mallocs == m0);
        bad = cfg;
        bad.P_adi[0] = 3;                                 // 16 % 3: refused by the sweep plan, nothing kept
        CHECK(ns_create(ctx, &bad, &ns) == TRI_E_SHAPE && !ns);
        CHECK(ns_create(ctx, &cfg, &ns) == TRI_OK && ns);
        std::vector<double> uu(nz * ny * (nx + 1)), vv(nz * (ny + 1) * nx), ww(nz * ny * nx), pp(nz * ny * nx);
        const int l0 = g_launches, m1 = g_mallocs, s0 = g_syncs;
        CHECK(ns_step(ns, uu.data(), vv.data(), ww.data(), pp.data()) == TRI_OK);
        CHECK(g_launches > l0 && g_mallocs == m1 && g_syncs == s0);
        REFUSED(ns_step(ns, uu.data(), vv.data(), ww.data(), ww.data()), TRI_E_ARG, ww);   // p over w
        REFUSED(ns_step(ns, uu.data(), nullptr, ww.data(), pp.data()), TRI_E_ARG, ww);
        CHECK(ns_step(nullptr, uu.data(), vv.data(), ww.data(), pp.data()) == TRI_E_ARG);
        CHECK(ns_destroy(ns) == TRI_OK);
    }

    CHECK(tri_destroy(ctx) == TRI_OK);
    CHECK(g_mallocs == g_frees);      // everything the library allocated was released
    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("api sanitizer driver: ok (%d launches)\n", g_launches);
    return 0;
}
