"""Host-side checks of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer: the library's host code (argument validation,
range checks, dispatch) is compiled with the sanitizers on its host pass
(the device code is built normally and never launched) and driven by a small
C program through every entry point with arguments that must be rejected
before any launch.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _gpu_present() -> bool:
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:  # pragma: no cover
        return False


pytestmark = pytest.mark.skipif(_gpu_present() or not os.path.exists(os.path.join(ROCM, "bin", "hipcc")),
                                reason="host sanitizer build runs on hosts without a GPU")

DRIVER = r"""
#include <stdio.h>
#include <stdint.h>
#include "eig3.h"
#define P(x) ((void *)(uintptr_t)(x))
static int fails = 0;
static void expect(int got, int want, const char *what) {
    if (got != want) { printf("FAIL %s: %d != %d\n", what, got, want); ++fails; }
}
int main(void) {
    eig3_matrices m = {0};
    m.n = 1024; m.dtype = EIG3_F64; m.structure = EIG3_GENERAL; m.layout = EIG3_SOA; m.accuracy = EIG3_FMA;
    for (int j = 0; j < 9; ++j) m.a[j] = (const void *)(uintptr_t)(0x20000000 + j * 1024 * 8);
    void *e27[27];
    for (int j = 0; j < 26; ++j) e27[j] = P(0x40000000 + j * 0x100000);
    e27[26] = (void *)m.a[3];
    expect(eig3_eigenprojectors(&m, EIG3_SOA, e27, NULL), EIG3_EINVAL, "projectors alias last slot");
    void *lam[3] = {P(0x50000000), P(0x50000000 + 8), P(0x51000000)};
    expect(eig3_eigvals(&m, EIG3_SOA, lam, NULL), EIG3_EINVAL, "eigvals outputs overlap");
    void *g[3] = {P(0x52000000), P(0x53000000), P(0x54000000)};
    void *gr[9];
    for (int j = 0; j < 9; ++j) gr[j] = P(0x60000000 + j * 0x100000);
    gr[8] = g[1];
    expect(eig3_eigvals_backward(&m, EIG3_SOA, (const void *const *)g, gr, NULL), EIG3_EINVAL, "grad aliases g");
    void *df[9];
    for (int j = 0; j < 9; ++j) df[j] = P(0x70000000 + j * 0x100000);
    df[8] = P(0x7F000000);
    expect(eig3_mohr_coulomb(&m, 100.0, 10.0, P(0x7F000000), df, NULL), EIG3_EINVAL, "dfds aliases f");
    expect(eig3_mohr_coulomb(&m, -1.0, 10.0, P(0x7F000000), NULL, NULL), EIG3_EINVAL, "bad s_yc");
    expect(eig3_invariants(&m, P(0x50000000), P(0x51000000), P(0x52000000), (void *)m.a[8], NULL), EIG3_EINVAL,
           "invariants alias input");
    void *fo[9];
    for (int j = 0; j < 9; ++j) fo[j] = P(0x78000000 + j * 0x100000);
    expect(eig3_matrix_function(&m, 7, fo, NULL), EIG3_EINVAL, "unknown matrix function");
    fo[4] = (void *)m.a[0];
    expect(eig3_matrix_function(&m, EIG3_EXP, fo, NULL), EIG3_EINVAL, "matrix function aliases input");
    m.n = -5;
    expect(eig3_eigvals(&m, EIG3_SOA, lam, NULL), EIG3_EINVAL, "n < 0");
    m.n = 0;
    expect(eig3_eigvals(&m, EIG3_SOA, lam, NULL), EIG3_OK, "n == 0");
    m.n = 1024; m.accuracy = 7;
    expect(eig3_eigvals(&m, EIG3_SOA, lam, NULL), EIG3_EINVAL, "bad accuracy");
    m.accuracy = EIG3_NAIVE; m.layout = EIG3_AOS; m.a[0] = P(0x20000004);
    expect(eig3_eigvals(&m, EIG3_AOS, lam, NULL), EIG3_EINVAL, "misaligned aos");
    printf("%s\n", fails ? "FAILED" : "ALL OK");
    return fails != 0;
}
"""


def test_host_code_under_sanitizers(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = shutil.which("clang") or pytest.skip("no clang")
    src = os.path.join(ROOT, "paper_2511_00292_amd", "csrc", "eig3.hip")
    lib = os.path.join(tmp_path, "libeig3_san.so")
    # each sanitizer flag applies to the host compilation only (the device
    # code is built normally and never launched here)
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all",
                    "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(ROOT, "include"), src, "-o", lib],
                   check=True, capture_output=True)
    drv = os.path.join(tmp_path, "driver.c")
    with open(drv, "w") as f:
        f.write(DRIVER)
    exe = os.path.join(tmp_path, "driver")
    subprocess.run([clang, "-g", "-fsanitize=address,undefined", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), drv,
                    lib, f"-Wl,-rpath,{tmp_path}", "-o", exe], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr
