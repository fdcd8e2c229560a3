/*
 * host_selftest.c -- drives the host side of librt3d.so's C ABI (argument
 * checks, defaults, null handling, context creation where a GPU exists) for
 * builds whose host code carries AddressSanitizer and UndefinedBehavior
 * Sanitizer (build.build_sanitized).  Exit status 0 when every call returns
 * what rt3d.h promises.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "../../include/rt3d.h"

static int failures = 0;

static void expect(int cond, const char* what)
{
    if (!cond) {
        fprintf(stderr, "host_selftest: %s\n", what);
        ++failures;
    }
}

int main(void)
{
    rt3d_params p;
    rt3d_params_default(&p);
    expect(p.struct_size == sizeof p && p.n_iter == 20 && p.k_max == 4, "defaults");
    rt3d_ctx* c = NULL;
    const double irf[3] = {1.0, 2.0, 1.0}, zero[2] = {0.0, 0.0}, neg[2] = {1.0, -1.0};
    const double nan2[2] = {1.0, NAN};
    expect(rt3d_create(zero, 2, -1, 100, &p, &c) == RT3D_E_INVALID, "zero-sum IRF");
    expect(rt3d_create(neg, 2, -1, 100, &p, &c) == RT3D_E_INVALID, "negative IRF sample");
    expect(rt3d_create(nan2, 2, -1, 100, &p, &c) == RT3D_E_INVALID, "non-finite IRF sample");
    expect(rt3d_create(irf, 3, -1, 2, &p, &c) == RT3D_E_INVALID, "IRF longer than the histogram");
    expect(rt3d_create(irf, 3, -1, 70000, &p, &c) == RT3D_E_INVALID, "bins above 65535");
    expect(rt3d_create(irf, 3, 3, 100, &p, &c) == RT3D_E_INVALID, "origin outside the IRF");
    expect(rt3d_create(NULL, 3, -1, 100, &p, &c) == RT3D_E_INVALID, "null IRF");
    expect(rt3d_create(irf, 3, -1, 100, NULL, &c) == RT3D_E_INVALID, "null params");
    rt3d_params bad = p;
    bad.k_max = 5;
    expect(rt3d_create(irf, 3, -1, 100, &bad, &c) == RT3D_E_INVALID, "k_max above the slot capacity");
    bad = p;
    bad.h_apss = 0.0;
    expect(rt3d_create(irf, 3, -1, 100, &bad, &c) == RT3D_E_INVALID, "zero APSS support");
    bad = p;
    bad.struct_size = 8;
    expect(rt3d_create(irf, 3, -1, 100, &bad, &c) == RT3D_E_INVALID, "struct_size");
    bad = p;
    bad.denoiser = 7;
    expect(rt3d_create(irf, 3, -1, 100, &bad, &c) == RT3D_E_UNSUPPORTED, "unknown denoiser");
    expect(c == NULL, "no context from a refused create");
    rt3d_destroy(NULL);
    expect(strcmp(rt3d_last_error(NULL), "null context") == 0, "last_error(NULL)");
    expect(rt3d_query(NULL, NULL, NULL) == RT3D_E_INVALID, "query(NULL)");
    expect(rt3d_workspace_bytes(NULL, 1, 1, 1, 1) == 0, "workspace_bytes(NULL)");
    expect(rt3d_denoiser_save(NULL, "x") == RT3D_E_INVALID, "denoiser_save(NULL)");
    expect(rt3d_denoiser_load(NULL, "x") == RT3D_E_INVALID, "denoiser_load(NULL)");
    expect(rt3d_compact_noalloc(NULL, NULL, 1, NULL, NULL, 1, NULL, NULL) == RT3D_E_INVALID, "compact_noalloc(NULL)");
    /* a valid create: a context with a GPU, E_DEVICE without one */
    const rt3d_status s = rt3d_create(irf, 3, -1, 100, &p, &c);
    expect(s == RT3D_OK || s == RT3D_E_DEVICE, "valid create");
    if (s == RT3D_OK) {
        expect(rt3d_workspace_bytes(c, 2, 8, 8, 1000) > 0, "workspace size");
        expect(rt3d_compact_noalloc(c, NULL, 1, NULL, NULL, 1, NULL, NULL) == RT3D_E_INVALID, "noalloc nulls");
        expect(rt3d_denoiser_save(c, "x") == RT3D_E_STATE, "save without the learned denoiser");
        rt3d_destroy(c);
    }
    printf("host_selftest: %s (create with valid arguments: %d)\n", failures ? "FAILED" : "ok", (int)s);
    return failures ? 1 : 0;
}
