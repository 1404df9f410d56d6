/* Host-side calls of the C ABI, for a build of the library's host code under
 * AddressSanitizer and UndefinedBehaviorSanitizer (no device code: nothing
 * here launches a kernel or touches a device).  Covers the plan and workspace
 * layout over every feature width, storage type, form, primitive and view
 * count, the tuning candidates, the buffer views, the size queries, and the
 * argument validation of every entry point.  Exit status 0 when every check
 * holds; the sanitizers abort on the first finding. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "fhgs.h"

static int failures = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            fprintf(stderr, "check failed (line %d): %s\n", __LINE__, #c);       \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

static fh_camera camera(int w, int h) {
    fh_camera c;
    memset(&c, 0, sizeof c);
    c.width = w;
    c.height = h;
    c.fx = c.fy = 0.8f * (float)w;
    c.cx = 0.5f * (float)w;
    c.cy = 0.5f * (float)h;
    c.R[0] = c.R[4] = c.R[8] = 1.0f;
    c.t[2] = 4.0f;
    return c;
}

/* workspace sub-buffers: 256-byte aligned, ascending, inside ws_bytes */
static void check_layout(const fh_plan *p) {
    CHECK(p->n_ws > 0 && p->n_ws <= FH_WS_SLOTS);
    for (int i = 0; i < p->n_ws; ++i) {
        CHECK(p->off[i] % 256 == 0);
        CHECK(p->off[i] <= p->ws_bytes);
        if (i > 0) CHECK(p->off[i] >= p->off[i - 1]);
    }
    CHECK(p->n_tiles == p->tile_off[p->n_views]);
    CHECK(p->n_pixels == p->pix_off[p->n_views]);
}

static void check_buffers(const fh_plan *p) {
    /* buffer views are offsets into the workspace; nothing is dereferenced */
    static unsigned char fake_ws[16];
    for (int b = FH_BUF_RECORDS; b <= FH_BUF_GRAD2D; ++b) {
        void *ptr = NULL;
        int64_t count = -1;
        CHECK(fh_get_buffer(p, fake_ws, (fh_buffer)b, &ptr, &count) == FH_OK);
        CHECK(count >= 0);
        CHECK((unsigned char *)ptr >= fake_ws && (size_t)((unsigned char *)ptr - fake_ws) <= p->ws_bytes);
    }
    void *ptr;
    int64_t count;
    CHECK(fh_get_buffer(p, fake_ws, (fh_buffer)99, &ptr, &count) == FH_E_INVALID);
    CHECK(fh_get_buffer(p, NULL, FH_BUF_RANGES, &ptr, &count) == FH_E_INVALID);
}

static void check_tuning(const fh_plan *p) {
    fh_tuning out[64];
    for (int which = FH_K_PROJECT; which <= FH_K_NDFD; ++which) {
        int32_t n = -1;
        CHECK(fh_tuning_candidates(p, which, out, 64, &n) == FH_OK);
        CHECK(n >= 1 && n <= 64);
        n = -1;
        CHECK(fh_tuning_candidates(p, which, out, 1, &n) == FH_OK);   /* truncated to max */
        CHECK(n == 1);
    }
    int32_t n;
    CHECK(fh_tuning_candidates(p, FH_K_RENDER_FWD, out, 0, &n) == FH_E_INVALID);
}

int main(void) {
    CHECK(fh_version() == FH_VERSION);
    for (int s = -9; s <= 3; ++s) CHECK(fh_status_string((fh_status)s) != NULL);

    fh_camera cams[FH_MAX_VIEWS];
    for (int i = 0; i < FH_MAX_VIEWS; ++i) cams[i] = camera(48 + 24 * (i % 5) + (i % 3), 40 + 16 * (i % 4) + (i % 7));

    static const int32_t widths[] = {0, 1, 8, 16, 32, 40, 64, 96, 128, 200, 256, 384, 512, 1024, 1025};
    static const int32_t views[] = {1, 3, 16, FH_MAX_VIEWS, FH_MAX_VIEWS + 1};
    static const int64_t ns[] = {0, 1, 1000, 3000000};
    int ok_plans = 0;
    for (size_t wi = 0; wi < sizeof widths / sizeof widths[0]; ++wi)
        for (int dt = FH_F32; dt <= FH_BF16; ++dt)
            for (int form = FH_FORM_F32; form <= FH_FORM_BF16; ++form)
                for (size_t vi = 0; vi < sizeof views / sizeof views[0]; ++vi)
                    for (size_t ni = 0; ni < sizeof ns / sizeof ns[0]; ++ni) {
                        fh_plan plan;
                        memset(&plan, 0xA5, sizeof plan);   /* no field may be read before it is set */
                        const fh_status st = fh_plan_init(&plan, ns[ni], 3, widths[wi], (fh_dtype)dt, (fh_form)form,
                                                          cams, views[vi], 40 * ns[ni] + 7, 4 * ns[ni] + 3);
                        if (views[vi] > FH_MAX_VIEWS || widths[wi] > 1024) CHECK(st != FH_OK);
                        if (st != FH_OK) {
                            CHECK(st == FH_E_INVALID || st == FH_E_UNSUPPORTED);
                            continue;
                        }
                        ++ok_plans;
                        check_layout(&plan);
                        check_tuning(&plan);
                        check_buffers(&plan);
                        for (int prim = FH_PRIM_GAUSSIAN; prim <= FH_PRIM_SURFEL; ++prim) {
                            const fh_status sp = fh_plan_set_primitive(&plan, prim);
                            CHECK(sp == FH_OK || sp == FH_E_UNSUPPORTED);
                            for (int nd = 1; nd >= 0; --nd) {
                                const fh_status sn = fh_plan_set_ndfd(&plan, nd);
                                CHECK(sn == FH_OK || sn == FH_E_UNSUPPORTED);
                                check_layout(&plan);
                                check_tuning(&plan);
                            }
                        }
                        CHECK(fh_plan_set_primitive(&plan, 2) == FH_E_INVALID);
                        CHECK(fh_plan_set_primitive(&plan, -1) == FH_E_INVALID);
                    }
    CHECK(ok_plans > 100);

    /* invalid plan arguments */
    fh_plan plan;
    CHECK(fh_plan_init(NULL, 10, 3, 16, FH_F32, FH_FORM_F32, cams, 1, 100, 100) == FH_E_INVALID);
    CHECK(fh_plan_init(&plan, -1, 3, 16, FH_F32, FH_FORM_F32, cams, 1, 100, 100) == FH_E_INVALID);
    CHECK(fh_plan_init(&plan, 10, 3, -1, FH_F32, FH_FORM_F32, cams, 1, 100, 100) == FH_E_INVALID);
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, FH_FORM_F32, NULL, 1, 100, 100) == FH_E_INVALID);
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, FH_FORM_F32, cams, 0, 100, 100) == FH_E_INVALID);
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, FH_FORM_F32, cams, 1, -1, 100) == FH_E_INVALID);
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, FH_FORM_F32, cams, 1, 100, -1) == FH_E_INVALID);
    CHECK(fh_plan_init(&plan, 10, 4, 16, FH_F32, FH_FORM_F32, cams, 1, 100, 100) == FH_E_UNSUPPORTED);
    CHECK(fh_plan_init(&plan, 10, -1, 16, FH_F32, FH_FORM_F32, cams, 1, 100, 100) != FH_OK);
    CHECK(fh_plan_init(&plan, 10, 3, 16, (fh_dtype)7, FH_FORM_F32, cams, 1, 100, 100) != FH_OK);
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, (fh_form)7, cams, 1, 100, 100) != FH_OK);
    fh_camera bad[2] = {camera(64, 48), camera(0, 48)};
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, FH_FORM_F32, bad, 2, 100, 100) != FH_OK);
    bad[1] = camera(64, -3);
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, FH_FORM_F32, bad, 2, 100, 100) != FH_OK);
    /* capacities whose workspace would not fit in size_t */
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, FH_FORM_F32, cams, 1, INT64_MAX / 2, 100) != FH_OK);
    CHECK(fh_plan_init(&plan, 10, 3, 16, FH_F32, FH_FORM_F32, cams, 1, 100, INT64_MAX / 4) != FH_OK);
    CHECK(fh_plan_init(&plan, INT64_MAX / 8, 3, 16, FH_F32, FH_FORM_F32, cams, 1, 100, 100) != FH_OK);
    CHECK(fh_plan_set_ndfd(NULL, 1) == FH_E_INVALID);
    CHECK(fh_plan_set_primitive(NULL, 1) == FH_E_INVALID);

    /* argument validation of the device entry points: rejected on the host,
     * before any launch */
    CHECK(fh_plan_init(&plan, 100, 3, 16, FH_F32, FH_FORM_F32, cams, 1, 5000, 1000) == FH_OK);
    static unsigned char fake_ws[16];
    fh_image img;
    memset(&img, 0, sizeof img);
    fh_counters cnt;
    uint64_t keys[1];
    uint32_t gids[1];
    CHECK(fh_project(NULL, NULL, NULL, 0) == FH_E_INVALID);
    CHECK(fh_project(&plan, NULL, fake_ws, 0) == FH_E_INVALID);
    CHECK(fh_bin_count(NULL, fake_ws, 0) == FH_E_INVALID);
    CHECK(fh_bin_sort(&plan, NULL, 0) == FH_E_INVALID);
    CHECK(fh_bin_keys(&plan, fake_ws, keys, gids, -1, 0) == FH_E_INVALID);
    CHECK(fh_bin_keys(&plan, fake_ws, keys, gids, plan.inst_capacity + 1, 0) == FH_E_INVALID);
    CHECK(fh_render_fwd(&plan, NULL, fake_ws, &img, 0) == FH_E_INVALID);
    CHECK(fh_render_bwd(&plan, NULL, fake_ws, &img, NULL, NULL, FH_F32, NULL, NULL, 0) == FH_E_INVALID);
    CHECK(fh_ndfd_losses(&plan, NULL, fake_ws, &img, NULL, 0.5f, 20.0f, NULL, NULL, 0) == FH_E_INVALID);
    CHECK(fh_fuse_features(&plan, NULL, fake_ws, &img, NULL, FH_BF16, NULL, 0) == FH_E_INVALID);
    CHECK(fh_fuse_finalize(NULL, 10, 16, NULL, NULL, FH_F32, 0) == FH_E_INVALID);
    CHECK(fh_read_counters(&plan, NULL, &cnt, 0) == FH_E_INVALID);
    CHECK(fh_get_status(&plan, fake_ws, NULL, 0) == FH_E_INVALID);
    CHECK(fh_render_fwd_static(&plan, NULL, &img, &cnt, 0) == FH_E_INVALID);
    CHECK(fh_autotune(&plan, NULL, NULL, &img, NULL, NULL, FH_F32, NULL, NULL, 1, 0) == FH_E_INVALID);
    CHECK(fh_set_kernel_events(FH_K_PROJECT, NULL, NULL, 2) == FH_E_INVALID);
    CHECK(fh_set_kernel_events((fh_kernel)99, NULL, NULL, 0) == FH_E_INVALID);
    CHECK(fh_set_kernel_events(FH_K_RENDER_BWD, NULL, NULL, 0) == FH_OK);   /* clears the hooks */
    CHECK(fh_adam_step(-1, 3, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0) == FH_E_INVALID);
    CHECK(fh_activate(-1, NULL, NULL, NULL, NULL, 0) == FH_E_INVALID);
    CHECK(fh_densify_stats(&plan, NULL, NULL, NULL, 0) == FH_E_INVALID);
    CHECK(fh_densify_plan(-1, NULL, NULL, NULL, 0, NULL, NULL, NULL, 0) == FH_E_INVALID);
    CHECK(fh_photometric_loss(0, NULL, NULL, NULL, NULL, NULL, 0) == FH_E_INVALID);

    /* size queries */
    CHECK(fh_densify_workspace_size(0) > 0);
    CHECK(fh_densify_workspace_size(3000000) > fh_densify_workspace_size(1000));
    CHECK(fh_loss_workspace_size(1) > 0);
    CHECK(fh_loss_workspace_size(1 << 24) >= fh_loss_workspace_size(1 << 10));

    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host calls: %d plans checked\n", ok_plans);
    return 0;
}
