/*
 * A plain C99 client of the nsasm C ABI (test helper): no C++, Python or
 * torch.  It reads a mesh and nodal fields from raw little-endian files in a
 * directory, builds the mesh, converts the fields to mesh order, assembles the
 * FP64 right-hand side and the velocity vector-Jacobian product, converts both
 * back to user order and writes them next to the inputs.
 *
 *   nsasm_client DIR N_NODES N_ELEMS
 *   inputs : DIR/coords.bin (f64 Nn x 3), conn.bin (i32 Ne x 4), u.bin (f64
 *            Nn x 3), p.bin (f64 Nn), lam.bin (f64 Nn x 3), params.bin (f64:
 *            rho, mu, cs, f0, f1, f2)
 *   outputs: DIR/rhs.bin, DIR/grad.bin (f64 Nn x 3)
 * Exit status 0 on success; otherwise a message on stderr.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "nsasm.h"

#define FAIL_HIP(call)                                                              \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));       \
            return 1;                                                               \
        }                                                                           \
    } while (0)

#define FAIL_NS(call)                                                               \
    do {                                                                            \
        nsasm_status s_ = (call);                                                   \
        if (s_ != NSASM_OK) {                                                       \
            fprintf(stderr, "%s returned %d: %s\n", #call, (int)s_, nsasm_last_error()); \
            return 1;                                                               \
        }                                                                           \
    } while (0)

static int read_file(const char *dir, const char *name, void *buf, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        return 1;
    }
    size_t got = fread(buf, 1, bytes, f);
    fclose(f);
    if (got != bytes) {
        fprintf(stderr, "%s: expected %zu bytes, read %zu\n", path, bytes, got);
        return 1;
    }
    return 0;
}

static int write_file(const char *dir, const char *name, const void *buf, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(buf, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", path);
        if (f) fclose(f);
        return 1;
    }
    fclose(f);
    return 0;
}

int main(int argc, char **argv) {
    if (argc != 4) {
        fprintf(stderr, "usage: %s DIR N_NODES N_ELEMS\n", argv[0]);
        return 2;
    }
    const char *dir = argv[1];
    const int64_t nn = atoll(argv[2]), ne = atoll(argv[3]);
    if (nn <= 0 || ne <= 0) {
        fprintf(stderr, "sizes must be positive\n");
        return 2;
    }
    const size_t vec = sizeof(double) * 3 * (size_t)nn, sca = sizeof(double) * (size_t)nn;
    const size_t cbytes = sizeof(int32_t) * 4 * (size_t)ne;
    double *coords = malloc(vec), *u = malloc(vec), *p = malloc(sca), *lam = malloc(vec), *out = malloc(vec);
    int32_t *conn = malloc(cbytes);
    double pv[6];
    if (!coords || !u || !p || !lam || !out || !conn) {
        fprintf(stderr, "out of host memory\n");
        return 1;
    }
    if (read_file(dir, "coords.bin", coords, vec) || read_file(dir, "conn.bin", conn, cbytes) ||
        read_file(dir, "u.bin", u, vec) || read_file(dir, "p.bin", p, sca) || read_file(dir, "lam.bin", lam, vec) ||
        read_file(dir, "params.bin", pv, sizeof pv))
        return 1;

    double *d_coords, *d_u, *d_p, *d_lam, *d_um, *d_pm, *d_lm, *d_res, *d_user;
    int32_t *d_conn;
    FAIL_HIP(hipMalloc((void **)&d_coords, vec));
    FAIL_HIP(hipMalloc((void **)&d_conn, cbytes));
    FAIL_HIP(hipMalloc((void **)&d_u, vec));
    FAIL_HIP(hipMalloc((void **)&d_p, sca));
    FAIL_HIP(hipMalloc((void **)&d_lam, vec));
    FAIL_HIP(hipMalloc((void **)&d_um, vec));
    FAIL_HIP(hipMalloc((void **)&d_pm, sca));
    FAIL_HIP(hipMalloc((void **)&d_lm, vec));
    FAIL_HIP(hipMalloc((void **)&d_res, vec));
    FAIL_HIP(hipMalloc((void **)&d_user, vec));
    FAIL_HIP(hipMemcpy(d_coords, coords, vec, hipMemcpyHostToDevice));
    FAIL_HIP(hipMemcpy(d_conn, conn, cbytes, hipMemcpyHostToDevice));
    FAIL_HIP(hipMemcpy(d_u, u, vec, hipMemcpyHostToDevice));
    FAIL_HIP(hipMemcpy(d_p, p, sca, hipMemcpyHostToDevice));
    FAIL_HIP(hipMemcpy(d_lam, lam, vec, hipMemcpyHostToDevice));

    nsasm_mesh *mesh = NULL;
    FAIL_NS(nsasm_mesh_create(d_coords, nn, d_conn, ne, NULL, NULL, &mesh));
    nsasm_params prm;
    memset(&prm, 0, sizeof prm);
    prm.rho = pv[0];
    prm.mu = pv[1];
    prm.smagorinsky_cs = pv[2];
    prm.body_force[0] = pv[3];
    prm.body_force[1] = pv[4];
    prm.body_force[2] = pv[5];
    prm.eddy_model = NSASM_EDDY_SMAGORINSKY;
    prm.convective_form = NSASM_CONVECTIVE_ADVECTIVE;

    FAIL_NS(nsasm_to_mesh_order(mesh, 3, NSASM_FP64, d_u, d_um, NULL));
    FAIL_NS(nsasm_to_mesh_order(mesh, 1, NSASM_FP64, d_p, d_pm, NULL));
    FAIL_NS(nsasm_to_mesh_order(mesh, 3, NSASM_FP64, d_lam, d_lm, NULL));

    FAIL_NS(nsasm_assemble_rhs(mesh, &prm, NSASM_FP64, d_um, d_pm, d_res, NULL));
    FAIL_NS(nsasm_from_mesh_order(mesh, 3, NSASM_FP64, d_res, d_user, NULL));
    FAIL_HIP(hipMemcpy(out, d_user, vec, hipMemcpyDeviceToHost));
    if (write_file(dir, "rhs.bin", out, vec)) return 1;

    FAIL_NS(nsasm_assemble_rhs_vjp(mesh, &prm, NSASM_FP64, d_um, d_lm, d_res, NULL));
    FAIL_NS(nsasm_from_mesh_order(mesh, 3, NSASM_FP64, d_res, d_user, NULL));
    FAIL_HIP(hipMemcpy(out, d_user, vec, hipMemcpyDeviceToHost));
    if (write_file(dir, "grad.bin", out, vec)) return 1;

    FAIL_NS(nsasm_mesh_destroy(mesh));
    hipFree(d_coords);
    hipFree(d_conn);
    hipFree(d_u);
    hipFree(d_p);
    hipFree(d_lam);
    hipFree(d_um);
    hipFree(d_pm);
    hipFree(d_lm);
    hipFree(d_res);
    hipFree(d_user);
    free(coords);
    free(u);
    free(p);
    free(lam);
    free(out);
    free(conn);
    printf("nsasm_client: %s, %lld nodes, %lld elements: ok\n", nsasm_version(), (long long)nn, (long long)ne);
    return 0;
}
