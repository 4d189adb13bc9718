/* Plain-C client of libsnn.so: include/snn.h must compile as C11, and the
 * host calibration routines run without a GPU.  Prints the fitted k1 k2 k3,
 * the MAPE and the picked runs; exits non-zero on an unexpected status. */
#include <math.h>
#include <stdio.h>

#include "snn.h"

int main(void)
{
    /* points on gScale = 1318 / (109.9 + nConn) - 0.28 (Table 1), nConn 100..1000 step 50 */
    double x[19], y[19], k[3], mape = -1.0;
    for (int i = 0; i < 19; ++i) {
        x[i] = 100.0 + 50.0 * i;
        y[i] = 1318.0 / (109.9 + x[i]) - 0.28;
    }
    int rc = snn_gscale_fit(19, x, y, k, &mape);
    if (rc != SNN_OK) {
        fprintf(stderr, "fit failed: %d %s\n", rc, snn_last_error());
        return 1;
    }
    printf("%.12g %.12g %.12g %.3g\n", k[0], k[1], k[2], mape);

    /* too few distinct nConn: SNN_EINVAL with a message */
    double x2[3] = {1.0, 1.0, 2.0}, y2[3] = {1.0, 1.0, 1.0};
    rc = snn_gscale_fit(3, x2, y2, k, NULL);
    if (rc != SNN_EINVAL || snn_last_error()[0] == '\0') return 2;

    /* Fig. 1 selection on a four-run table, reference run 0 */
    double n_conn[4] = {10.0, 20.0, 20.0, 20.0}, gs[4] = {1.0, 0.5, 0.25, 2.0};
    double avg[4] = {5.0, 5.5, 4.0, 5.0};
    int32_t nans[4] = {0, 0, 0, 7};
    int64_t n_groups = 0, picked[4];
    double groups[4];
    rc = snn_gscale_select(4, n_conn, gs, avg, nans, 0, &n_groups, groups, picked);
    if (rc != SNN_OK) return 3;
    printf("%lld %g %lld %g %lld\n", (long long)n_groups, groups[0], (long long)picked[0], groups[1],
           (long long)picked[1]);
    return 0;
}
