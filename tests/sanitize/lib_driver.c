/* Drives the host-side logic of liblddmm -- argument validation, workspace
 * sizing, status strings, error reporting -- in a build whose host code
 * carries AddressSanitizer and UndefinedBehaviorSanitizer.  Every call here
 * either needs no device or is rejected before one is touched; a plan
 * creation on a machine without a GPU must fail with EDEVICE and no leak.
 * Exit status 0 when every call returned what the header promises. */
#include <stdio.h>
#include <string.h>

#include "../../include/lddmm.h"

static int fails = 0;

static void expect(int cond, const char *what)
{
    if (!cond) {
        printf("FAILED: %s (last error: %s)\n", what, lddmm_last_error());
        fails++;
    }
}

int main(int argc, char **argv)
{
    const int have_gpu = argc > 1 && strcmp(argv[1], "gpu") == 0;
    lddmm_config c = {{32, 24, 40}, 4, LDDMM_REG_H2S, 0, 0, 1e-3};
    size_t bytes = 0;
    expect(lddmm_workspace_bytes(&c, &bytes) == LDDMM_OK && bytes > 0, "workspace_bytes valid");
    expect(lddmm_workspace_bytes(NULL, &bytes) == LDDMM_EINVAL, "workspace_bytes NULL cfg");
    expect(lddmm_workspace_bytes(&c, NULL) == LDDMM_EINVAL, "workspace_bytes NULL out");
    const int bad_n[][3] = {{7, 8, 8}, {8, 14, 8}, {8, 8, 2048}, {0, 8, 8}, {-8, 8, 8}, {8, 8, 22}};
    for (unsigned i = 0; i < sizeof(bad_n) / sizeof(bad_n[0]); i++) {
        lddmm_config b = c;
        memcpy(b.n, bad_n[i], sizeof(b.n));
        expect(lddmm_workspace_bytes(&b, &bytes) == LDDMM_EINVAL, "bad grid rejected");
        lddmm_plan *p = (lddmm_plan *)1;
        expect(lddmm_plan_create(&b, NULL, &p) == LDDMM_EINVAL && p == NULL, "bad grid plan rejected");
        expect(strlen(lddmm_last_error()) > 0, "error detail set");
    }
    lddmm_config b = c;
    b.nt = 0;
    expect(lddmm_workspace_bytes(&b, &bytes) == LDDMM_EINVAL, "nt 0 rejected");
    b = c;
    b.beta = -1.0;
    expect(lddmm_workspace_bytes(&b, &bytes) == LDDMM_EINVAL, "negative beta rejected");
    b = c;
    b.reg = 3;
    expect(lddmm_workspace_bytes(&b, &bytes) == LDDMM_EINVAL, "bad reg rejected");
    b = c;
    b.flags = 64;
    expect(lddmm_workspace_bytes(&b, &bytes) == LDDMM_EINVAL, "bad flags rejected");
    b = c;
    b.n[0] = b.n[1] = 1024;
    b.n[2] = 1024;
    b.nt = 256;
    expect(lddmm_workspace_bytes(&b, &bytes) == LDDMM_OK && bytes > ((size_t)1 << 40), "huge workspace sized");
    for (int s = 0; s <= 7; s++) expect(lddmm_status_string((lddmm_status)s) != NULL, "status string");
    expect(lddmm_plan_create(&c, NULL, NULL) == LDDMM_EINVAL, "NULL plan out");
    expect(lddmm_plan_destroy(NULL) == LDDMM_EINVAL, "destroy NULL");
    expect(lddmm_set_images(NULL, NULL, NULL) == LDDMM_EINVAL, "set_images NULL plan");
    expect(lddmm_gradient(NULL, NULL, NULL) == LDDMM_EINVAL, "gradient NULL plan");
    expect(lddmm_transport_forward_static(NULL, NULL, NULL, NULL, NULL, NULL) == LDDMM_EINVAL,
           "static transport NULL cfg");
    lddmm_config big = c;
    big.n[0] = big.n[1] = big.n[2] = 256;
    float dummy[4] __attribute__((aligned(16)));
    expect(lddmm_transport_forward_static(&big, NULL, dummy, dummy, dummy + 0, NULL) == LDDMM_EINVAL,
           "static transport aliasing / size rejected");
    expect(lddmm_num_kernels() > 0 && lddmm_kernel_name(0) != NULL, "kernel names");
    lddmm_plan *p = NULL;
    const lddmm_status st = lddmm_plan_create(&c, NULL, &p);
    if (have_gpu) {
        expect(st == LDDMM_OK && p != NULL, "plan on a GPU");
        if (p) expect(lddmm_plan_destroy(p) == LDDMM_OK, "plan destroyed");
    } else {
        expect(st == LDDMM_EDEVICE && p == NULL, "plan without a GPU: EDEVICE");
    }
    printf(fails ? "library host sanitizer run: %d failures\n" : "library host sanitizer run: ok\n", fails);
    return fails ? 1 : 0;
}
