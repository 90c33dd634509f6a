/* A plain C99 client of libmpcd: only include/mpcd.h and the shared library,
 * no Python and no PyTorch.  The context uses its defaults (hipMalloc and a
 * stream of its own).  It checks the status codes of the boundary, admits a
 * Maxwell box, steps it, reads its diagnostics and state, writes a state
 * back and steps again, and prints "ok" or the first failed check.
 * Exit status: 0 ok, 1 a failed check, 77 no usable device. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpcd.h"

static int failed(const char* what, int rc)
{
    printf("FAILED %s: %d (%s)\n", what, rc, mpcd_strerror(rc));
    return 1;
}

int main(void)
{
    if (mpcd_abi_version() != MPCD_ABI_VERSION) return failed("abi version", mpcd_abi_version());
    mpcd_ctx* ctx = NULL;
    int rc = mpcd_create(NULL, &ctx);
    if (rc == MPCD_EDEVICE) {
        printf("no device\n");
        return 77;
    }
    if (rc != MPCD_OK) return failed("create", rc);

    const int32_t L = 12;
    const int64_t n = 10 * (int64_t)L * L * L;
    mpcd_box_desc d;
    memset(&d, 0, sizeof d);
    d.L[0] = d.L[1] = d.L[2] = L;
    d.a = 1.0;
    d.n_particles = n;
    d.dt = 0.1;
    d.alpha = 130.0 * 3.14159265358979323846 / 180.0;
    d.kT = 1.0;
    d.mass = 1.0;
    d.seed = 20221211u;
    d.flags = MPCD_INIT_MAXWELL | MPCD_TRACK_VACF;
    d.vacf_stride = 5;

    /* invalid arguments are refused without touching the context */
    int32_t slot = -1;
    mpcd_box_desc bad = d;
    bad.dt = -1.0;
    if ((rc = mpcd_admit(ctx, &bad, &slot)) != MPCD_EINVAL) return failed("admit bad dt", rc);
    mpcd_observables o;
    if ((rc = mpcd_observe(ctx, 3, &o)) != MPCD_ENOTFOUND) return failed("observe empty slot", rc);

    if ((rc = mpcd_admit(ctx, &d, &slot)) != MPCD_OK) return failed("admit", rc);
    if ((rc = mpcd_step(ctx, 20)) != MPCD_OK) return failed("step", rc);
    if ((rc = mpcd_observe(ctx, slot, &o)) != MPCD_OK) return failed("observe", rc);
    if (o.step != 20 || o.n_particles != n) return failed("observe step / n", (int)o.step);
    /* SRD conserves momentum (zero at the start) and energy exactly per cell */
    if (fabs(o.T - 1.0) > 1e-4) return failed("temperature after 20 steps", (int)(o.T * 1e6));
    for (int k = 0; k < 3; ++k)
        if (fabs(o.P[k]) > 1e-6 * (double)n) return failed("momentum", k);
    if (o.vacf_len != 5 || !o.vacf || fabs(o.vacf[0] - 3.0) > 0.05) return failed("vacf samples", o.vacf_len);

    float* s = (float*)malloc(sizeof(float) * 6 * (size_t)n);
    int64_t step = -1;
    if (!s) return failed("malloc", 0);
    if ((rc = mpcd_get_state(ctx, slot, s, &step)) != MPCD_OK || step != 20) return failed("get_state", rc);
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!(s[i] >= 0.0f && s[i] < (float)L)) return failed("position range", (int)i);
    /* a state written back is the state read back; the step counter too */
    if ((rc = mpcd_set_state(ctx, slot, s, 7)) != MPCD_OK) return failed("set_state", rc);
    float* t = (float*)malloc(sizeof(float) * 6 * (size_t)n);
    if (!t) return failed("malloc", 0);
    if ((rc = mpcd_get_state(ctx, slot, t, &step)) != MPCD_OK || step != 7) return failed("get_state 2", rc);
    if (memcmp(s, t, sizeof(float) * 6 * (size_t)n) != 0) return failed("state round trip", 0);
    s[0] = (float)L;   /* outside [0, L a): refused, state unchanged */
    if ((rc = mpcd_set_state(ctx, slot, s, 0)) != MPCD_EINVAL) return failed("set_state range", rc);
    if ((rc = mpcd_step(ctx, 3)) != MPCD_OK) return failed("step 2", rc);
    if ((rc = mpcd_observe(ctx, slot, &o)) != MPCD_OK || o.step != 10) return failed("observe 2", rc);

    mpcd_kernel_stat ks[16];
    int32_t nk = 0;
    if ((rc = mpcd_profile(ctx, 1)) != MPCD_OK) return failed("profile", rc);
    if ((rc = mpcd_step(ctx, 2)) != MPCD_OK) return failed("step 3", rc);
    if ((rc = mpcd_kernel_stats(ctx, ks, 16, &nk)) != MPCD_OK || nk < 1) return failed("kernel_stats", rc);

    if ((rc = mpcd_release(ctx, slot)) != MPCD_OK) return failed("release", rc);
    if ((rc = mpcd_release(ctx, slot)) != MPCD_ENOTFOUND) return failed("release twice", rc);
    mpcd_destroy(ctx);
    free(s);
    free(t);
    printf("ok\n");
    return 0;
}
