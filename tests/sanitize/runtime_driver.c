/* Drives the host side of libwdr's C ABI (include/wdr.h) through the paths
 * that need no GPU: status strings, defaults, geometry validation, null and
 * foreign arguments, a context request with no usable device.  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (no
 * device code) by tests/test_sanitize_cpu.py, which fails on any report.
 * Test infrastructure only. */
#include <stdio.h>
#include <string.h>

#include "../../include/wdr.h"

static int fails = 0;
#define EXPECT(cond)                                                                   \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            printf("FAIL %s:%d %s (%s)\n", __FILE__, __LINE__, #cond, wdr_last_error()); \
            ++fails;                                                                   \
        }                                                                              \
    } while (0)

static wdr_geom geom(int l, int b, int bc)
{
    wdr_geom g;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = l;
        g.B[mu] = b;
        g.bc[mu] = bc;
    }
    return g;
}

int main(void)
{
    for (int s = 1; s >= -6; --s) EXPECT(wdr_status_str((wdr_status)s) != NULL);
    wdr_solver_params sp;
    wdr_default_solver_params(&sp);
    EXPECT(sp.tol > 0 && sp.max_iter > 0);
    wdr_ctx *c = (wdr_ctx *)0x1;
    EXPECT(wdr_ctx_create(NULL, 0, &c) == WDR_EINVAL);
    wdr_geom g = geom(8, 3, 1);  /* odd block */
    EXPECT(wdr_ctx_create(&g, 0, &c) == WDR_EINVAL && c == NULL);
    g = geom(10, 4, 1);  /* B does not divide L */
    EXPECT(wdr_ctx_create(&g, 0, &c) == WDR_EINVAL);
    g = geom(8, 4, 2);  /* bc out of range */
    EXPECT(wdr_ctx_create(&g, 0, &c) == WDR_EINVAL);
    g = geom(512, 256, 1);  /* block too large */
    EXPECT(wdr_ctx_create(&g, 0, &c) == WDR_EINVAL);
    g = geom(8, 4, 1);  /* valid, but no usable device here */
    EXPECT(wdr_ctx_create(&g, 0, &c) != WDR_OK && c == NULL);
    EXPECT(wdr_ctx_create(&g, -1, &c) != WDR_OK);
    EXPECT(strlen(wdr_last_error()) > 0);
    EXPECT(wdr_ctx_destroy(NULL) == WDR_OK || wdr_ctx_destroy(NULL) == WDR_EINVAL);
    EXPECT(wdr_gauge_destroy(NULL) == WDR_OK);
    EXPECT(wdr_gauge_is_su3(NULL) == 0);
    EXPECT(wdr_ctx_volume(NULL) <= 0);
    (void)wdr_traffic(1);
    double buf[24];
    EXPECT(wdr_apply_D(NULL, NULL, 0.1, WDR_F64, buf, buf, NULL) == WDR_EINVAL);
    EXPECT(wdr_solve(NULL, NULL, 0.1, &sp, buf, buf, NULL, NULL) == WDR_EINVAL);
    EXPECT(wdr_gauge_set_clover(NULL, NULL, 1.0, 0.1, NULL) == WDR_EINVAL);
    EXPECT(wdr_clover_field(NULL, NULL, 0, buf, NULL) == WDR_EINVAL);
    EXPECT(wdr_logdet_ratio_batch(0, NULL, NULL, NULL, NULL, NULL, NULL) == WDR_EINVAL);
    wdr_est_params ep;
    memset(&ep, 0, sizeof(ep));
    EXPECT(wdr_logdet_ratio(NULL, NULL, NULL, 0.1, &ep, NULL, NULL, NULL, NULL) == WDR_EINVAL);
    printf("runtime driver: %d failures\n", fails);
    return fails ? 1 : 0;
}
