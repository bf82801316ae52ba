/*
 * A plain C caller of libeig3 (test program): device memory from hipMalloc,
 * its own stream, the C entry points of eig3.h, no Python or PyTorch.
 *
 *   c_caller <n> <a.bin> <g.bin> <lam.bin> <inv.bin> <grad.bin>
 *
 * a.bin: n general binary64 matrices, row-major (n, 9); g.bin: (n, 3).
 * The matrices go to the device as 9 structure-of-arrays columns (with the
 * gradient's 9, in one allocation at eig3_soa_stride), the
 * results come back as lam (n, 3), inv (n, 4: I1 J2 J3 Delta) and grad
 * (n, 9).  Exit status 0 on success; any HIP or eig3 error prints a message
 * and exits non-zero.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "eig3.h"

#define HIP_OK(call)                                                               \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));     \
            exit(3);                                                               \
        }                                                                          \
    } while (0)

#define EIG3_OK_CALL(call)                                                         \
    do {                                                                           \
        int s_ = (call);                                                           \
        if (s_ != EIG3_OK) {                                                       \
            fprintf(stderr, "%s returned %s\n", #call, eig3_status_string(s_));   \
            exit(4);                                                               \
        }                                                                          \
    } while (0)

static double *read_file(const char *path, size_t count)
{
    double *p = malloc(count * sizeof(double));
    FILE *f = fopen(path, "rb");
    if (!p || !f || fread(p, sizeof(double), count, f) != count) {
        fprintf(stderr, "cannot read %zu values from %s\n", count, path);
        exit(2);
    }
    fclose(f);
    return p;
}

static void write_file(const char *path, const double *p, size_t count)
{
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, sizeof(double), count, f) != count) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(2);
    }
    fclose(f);
}

int main(int argc, char **argv)
{
    if (argc != 7) {
        fprintf(stderr, "usage: c_caller n a.bin g.bin lam.bin inv.bin grad.bin\n");
        return 1;
    }
    const int64_t n = atoll(argv[1]);
    if (n <= 0)
        return 1;
    const size_t nn = (size_t)n, bytes = nn * sizeof(double);
    double *a = read_file(argv[2], nn * 9), *g = read_file(argv[3], nn * 3);
    double *col = malloc(bytes), *out = malloc(bytes * 9);
    if (!col || !out)
        return 2;

    hipStream_t stream;
    HIP_OK(hipStreamCreate(&stream));
    double *da[9], *dg[3], *dl[3], *di[4], *dgr[9];
    /* A and the gradient: 18 arrays in one allocation at the recommended
       stride; g, the eigenvalues and the invariants: separate allocations */
    const int64_t stride = eig3_soa_stride(n, EIG3_F64);
    if (stride < n) {
        fprintf(stderr, "eig3_soa_stride returned %lld\n", (long long)stride);
        return 3;
    }
    double *dbuf;
    HIP_OK(hipMalloc((void **)&dbuf, 18 * (size_t)stride * sizeof(double)));
    for (int k = 0; k < 9; ++k) {
        da[k] = dbuf + (size_t)k * (size_t)stride;
        dgr[k] = dbuf + (size_t)(9 + k) * (size_t)stride;
        for (size_t m = 0; m < nn; ++m)
            col[m] = a[9 * m + k];
        HIP_OK(hipMemcpy(da[k], col, bytes, hipMemcpyHostToDevice));
    }
    for (int k = 0; k < 3; ++k) {
        HIP_OK(hipMalloc((void **)&dg[k], bytes));
        HIP_OK(hipMalloc((void **)&dl[k], bytes));
        for (size_t m = 0; m < nn; ++m)
            col[m] = g[3 * m + k];
        HIP_OK(hipMemcpy(dg[k], col, bytes, hipMemcpyHostToDevice));
    }
    for (int k = 0; k < 4; ++k)
        HIP_OK(hipMalloc((void **)&di[k], bytes));

    eig3_matrices A;
    memset(&A, 0, sizeof A);
    A.n = n;
    A.dtype = EIG3_F64;
    A.structure = EIG3_GENERAL;
    A.layout = EIG3_SOA;
    A.accuracy = EIG3_DOUBLE_WORD;
    for (int k = 0; k < 9; ++k)
        A.a[k] = da[k];

    /* a rejected call launches nothing and reports why */
    eig3_matrices bad = A;
    bad.n = -1;
    if (eig3_eigvals(&bad, EIG3_SOA, (void *const *)dl, stream) != EIG3_EINVAL) {
        fprintf(stderr, "n < 0 was not rejected\n");
        return 5;
    }

    EIG3_OK_CALL(eig3_invariants(&A, di[0], di[1], di[2], di[3], stream));
    EIG3_OK_CALL(eig3_eigvals(&A, EIG3_SOA, (void *const *)dl, stream));
    EIG3_OK_CALL(eig3_eigvals_backward(&A, EIG3_SOA, (const void *const *)dg, (void *const *)dgr, stream));
    HIP_OK(hipStreamSynchronize(stream));

    /* interleave the structure-of-arrays results row by row */
    for (int k = 0; k < 3; ++k) {
        HIP_OK(hipMemcpy(col, dl[k], bytes, hipMemcpyDeviceToHost));
        for (size_t m = 0; m < nn; ++m)
            out[3 * m + k] = col[m];
    }
    write_file(argv[4], out, nn * 3);
    for (int k = 0; k < 4; ++k) {
        HIP_OK(hipMemcpy(col, di[k], bytes, hipMemcpyDeviceToHost));
        for (size_t m = 0; m < nn; ++m)
            out[4 * m + k] = col[m];
    }
    write_file(argv[5], out, nn * 4);
    for (int k = 0; k < 9; ++k) {
        HIP_OK(hipMemcpy(col, dgr[k], bytes, hipMemcpyDeviceToHost));
        for (size_t m = 0; m < nn; ++m)
            out[9 * m + k] = col[m];
    }
    write_file(argv[6], out, nn * 9);

    HIP_OK(hipFree(dbuf));
    for (int k = 0; k < 3; ++k) {
        HIP_OK(hipFree(dg[k]));
        HIP_OK(hipFree(dl[k]));
    }
    for (int k = 0; k < 4; ++k)
        HIP_OK(hipFree(di[k]));
    HIP_OK(hipStreamDestroy(stream));
    free(a);
    free(g);
    free(col);
    free(out);
    printf("c_caller ok: %lld matrices, library %s\n", (long long)n, eig3_version());
    return 0;
}
