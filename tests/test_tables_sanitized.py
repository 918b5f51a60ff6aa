"""The library's host table builder under AddressSanitizer and
UndefinedBehaviorSanitizer.

qed_tables.cpp is plain host C++ (the FP64 quadrature behind
qed_tables_compute_host).  It is compiled here with g++
-fsanitize=address,undefined next to a small driver that builds a reduced
table set and checks that every entry is finite and that the quantile rows
increase.  Any out-of-bounds access, data race on a freed buffer or
undefined behaviour aborts the driver.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "paper_1311_1107_amd", "csrc", "qed_tables.cpp")

DRIVER = r'''
#include <cmath>
#include <cstdio>
#include <vector>
namespace qedtab {
int build_tables(double e_chi_min, double e_chi_max, int e_n_chi, int e_n_q, double e_logit,
                 double p_chi_min, double p_chi_max, int p_n_chi, int p_n_q, double p_logit,
                 double *ln_hrad, double *ln_g, double *emit_q, double *pair_lnh, double *pair_q);
}
int main() {
    const int nc = 12, nq = 10;
    std::vector<double> a(nc), b(nc), c(nc * nq), d(nc), e(nc * nq);
    const int rc = qedtab::build_tables(1e-3, 1e2, nc, nq, 18.0, 1e-2, 1e2, nc, nq, 18.0,
                                        a.data(), b.data(), c.data(), d.data(), e.data());
    if (rc) { std::printf("build_tables returned %d\n", rc); return 2; }
    for (int i = 0; i < nc; ++i) {
        if (!std::isfinite(a[i]) || !std::isfinite(b[i]) || !std::isfinite(d[i])) return 3;
        for (int k = 1; k < nq; ++k)
            if (!(c[i * nq + k] > c[i * nq + k - 1]) || !(e[i * nq + k] > e[i * nq + k - 1])) return 4;
    }
    std::printf("tables ok %.6f %.6f\n", a[0], d[nc - 1]);
    return 0;
}
'''


def test_table_builder_runs_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not installed")
    drv = tmp_path / "driver.cpp"
    drv.write_text(DRIVER)
    exe = tmp_path / "tables_san"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-pthread", "-o", str(exe), str(drv), SRC]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("the sanitizer runtimes are not installed: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, (res.stdout + res.stderr)[-3000:]
    assert "tables ok" in res.stdout
