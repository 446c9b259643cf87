/* A plain C client of libsw2d: no C++ and no PyTorch, only the C ABI of include/sw2d.h and
 * the HIP runtime's C API for device memory and a stream, which the caller owns.
 *
 * usage: sw2d_client DIR NX NY DX DY G DT EPS NSTEPS STEPS_PER_PASS ROWS
 * Reads DIR/H.f32, DIR/mask.u8 and DIR/eta.f32 ([NY][NX] each; u = v = 0), advances NSTEPS
 * steps (STEPS_PER_PASS steps per pass on ROWS-row bands when above 1), writes the final
 * state to DIR/out_eta.f32, DIR/out_u.f32, DIR/out_v.f32 and prints the folds of the last
 * steps kept in the ring, one line per step: step vol_total vol_disp max_abs_u max_abs_v.
 * Exit status: 0, or 2 for a bad argument or file, or 10 + (-status) for a library error. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "sw2d.h"

static int read_file(const char *dir, const char *name, void *buf, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) return 0;
    const size_t got = fread(buf, 1, bytes, f);
    fclose(f);
    return got == bytes;
}

static int write_file(const char *dir, const char *name, const void *buf, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f) return 0;
    const size_t put = fwrite(buf, 1, bytes, f);
    return fclose(f) == 0 && put == bytes;
}

static int lib_fail(const char *what, int rc) {
    fprintf(stderr, "%s: %s (%d)\n", what, sw2d_strerror(rc), rc);
    return 10 - rc;
}

int main(int argc, char **argv) {
    if (argc != 12) {
        fprintf(stderr, "usage: %s DIR NX NY DX DY G DT EPS NSTEPS STEPS_PER_PASS ROWS\n", argv[0]);
        return 2;
    }
    const char *dir = argv[1];
    sw2d_params p = {0};
    p.nx = atoi(argv[2]);
    p.ny = atoi(argv[3]);
    p.dx = atof(argv[4]);
    p.dy = atof(argv[5]);
    p.g = atof(argv[6]);
    p.dt = atof(argv[7]);
    p.eps = atof(argv[8]);
    const int nsteps = atoi(argv[9]), spp = atoi(argv[10]), rows = atoi(argv[11]);
    if (p.nx < 1 || p.ny < 1 || nsteps < 0) return 2;
    const size_t n = (size_t)p.nx * p.ny;

    float *H = malloc(n * sizeof(float)), *state = calloc(6 * n, sizeof(float));
    uint8_t *mask = malloc(n);
    if (!H || !state || !mask) return 2;
    if (!read_file(dir, "H.f32", H, n * sizeof(float)) || !read_file(dir, "mask.u8", mask, n) ||
        !read_file(dir, "eta.f32", state, n * sizeof(float)))
        return 2;

    const size_t work_bytes = sw2d_workspace_bytes(&p);
    if (work_bytes == 0) return 2;
    float *d_H = NULL, *d_state = NULL;
    uint8_t *d_mask = NULL;
    void *d_work = NULL;
    hipStream_t stream = NULL;
    if (hipMalloc((void **)&d_H, n * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&d_mask, n) != hipSuccess ||
        hipMalloc((void **)&d_state, 6 * n * sizeof(float)) != hipSuccess ||
        hipMalloc(&d_work, work_bytes) != hipSuccess || hipStreamCreate(&stream) != hipSuccess ||
        hipMemcpy(d_H, H, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_mask, mask, n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_state, state, 6 * n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        fprintf(stderr, "HIP set-up failed\n");
        return 2;
    }

    sw2d_t h = NULL;
    int rc = sw2d_create(&p, d_H, d_mask, d_state, d_work, work_bytes, stream, &h);
    if (rc != SW2D_OK) return lib_fail("sw2d_create", rc);
    if (spp > 1 && (rc = sw2d_set_time_blocking(h, spp, rows)) != SW2D_OK)
        return lib_fail("sw2d_set_time_blocking", rc);
    if (spp <= 1 && rows > 0 && (rc = sw2d_set_band_rows(h, rows)) != SW2D_OK)
        return lib_fail("sw2d_set_band_rows", rc);
    if ((rc = sw2d_step(h, nsteps)) != SW2D_OK) return lib_fail("sw2d_step", rc);

    int k = nsteps < sw2d_ring_capacity() ? nsteps : sw2d_ring_capacity();
    sw2d_red *red = malloc((size_t)(k > 0 ? k : 1) * sizeof(sw2d_red));
    if (!red) return 2;
    if (k > 0 && (rc = sw2d_reduce(h, red, k)) != SW2D_OK) return lib_fail("sw2d_reduce", rc);
    float *d_e = NULL, *d_u = NULL, *d_v = NULL;
    if ((rc = sw2d_state(h, &d_e, &d_u, &d_v)) != SW2D_OK) return lib_fail("sw2d_state", rc);
    if (hipStreamSynchronize(stream) != hipSuccess ||
        hipMemcpy(state, d_e, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(state + n, d_u, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(state + 2 * n, d_v, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
        fprintf(stderr, "HIP copy-back failed\n");
        return 2;
    }
    if (!write_file(dir, "out_eta.f32", state, n * sizeof(float)) ||
        !write_file(dir, "out_u.f32", state + n, n * sizeof(float)) ||
        !write_file(dir, "out_v.f32", state + 2 * n, n * sizeof(float)))
        return 2;
    for (int i = 0; i < k; ++i)
        printf("%lld %.17g %.17g %.9g %.9g\n", (long long)red[i].step, red[i].vol_total, red[i].vol_disp,
               (double)red[i].max_abs_u, (double)red[i].max_abs_v);

    if ((rc = sw2d_destroy(h)) != SW2D_OK) return lib_fail("sw2d_destroy", rc);
    (void)hipStreamDestroy(stream);
    (void)hipFree(d_work);
    (void)hipFree(d_state);
    (void)hipFree(d_mask);
    (void)hipFree(d_H);
    free(red);
    free(mask);
    free(state);
    free(H);
    return 0;
}
