"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the tree method of the library (csrc/host_tree.cpp) and the C oracle
(oracle/oracle.c), each built with g++/gcc into a small driver that runs
them over every small size, split, thread count and argument error, with any
sanitizer report fatal.  No GPU code is built here."""
import os
import shutil
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="host compilers missing")

TREE_DRIVER = textwrap.dedent(r"""
    #include <cstdint>
    #include <cstdio>
    #include <cstring>
    #include <vector>
    #include "ptd.h"

    static uint64_t s = 88172645463325252ull;
    static double rnd() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (double)(s >> 11) / 9007199254740992.0 - 0.5; }

    int main()
    {
        for (int n = 1; n <= 6; ++n) {
            const int64_t N = 1 << n, lda = N + 3;  // a padded row pitch
            std::vector<double> A(2 * N * lda);
            for (auto& v : A) v = rnd();
            std::vector<double> ref(2 * N * N), got(2 * N * N);
            uint64_t ops = 0;
            if (ptd_host_tree_decompose(n, 0, A.data(), lda, ref.data(), 0, 0, 1, 1, &ops) != 0) return 1;
            for (int split = 0; split <= n && split <= 3; ++split)
                for (int threads = 1; threads <= 3; ++threads) {
                    std::fill(got.begin(), got.end(), 0.0);
                    const int64_t trees = (int64_t)1 << (2 * split);
                    // two ranges that together cover the forest
                    if (ptd_host_tree_decompose(n, 0, A.data(), lda, got.data(), split, 0, trees / 2, threads, nullptr))
                        return 2;
                    if (ptd_host_tree_decompose(n, 0, A.data(), lda, got.data(), split, trees / 2, trees, threads, nullptr))
                        return 3;
                    if (std::memcmp(got.data(), ref.data(), got.size() * sizeof(double)) != 0) return 4;
                }
            std::vector<double> d(2 * N * N, 0.0);
            if (ptd_host_tree_decompose(n, PTD_DIAGONAL, A.data(), lda, d.data(), n, 0, (int64_t)1 << n, 2, &ops))
                return 5;
            // argument errors return before touching memory
            if (ptd_host_tree_decompose(n, 1u, A.data(), lda, got.data(), 0, 0, 1, 1, nullptr) != PTD_EINVAL) return 6;
            if (ptd_host_tree_decompose(n, 0, A.data(), N - 1, got.data(), 0, 0, 1, 1, nullptr) != PTD_EINVAL) return 7;
            if (ptd_host_tree_decompose(n, 0, A.data(), lda, got.data(), n + 1, 0, 1, 1, nullptr) != PTD_EINVAL) return 8;
        }
        std::puts("tree ok");
        return 0;
    }
""")

ORACLE_DRIVER = textwrap.dedent(r"""
    #include <math.h>
    #include <stdint.h>
    #include <stdio.h>
    #include <stdlib.h>

    int oracle_decompose_f64(int n, const double *A, double *out, int nthreads);
    int oracle_decompose_i64(int n, const int64_t *A, int64_t *out, int nthreads);
    int oracle_coeffs_f64(int n, const double *A, int64_t count, const uint32_t *xs, const uint32_t *zs,
                          double *out, int nthreads);
    int oracle_rows_f64(int n, const double *A, int64_t count, const uint32_t *xs, double *out, int nthreads);
    int oracle_reconstruct_f64(int n, const double *coeff, double *A);

    int main(void)
    {
        uint64_t s = 2463534242u;
        for (int n = 1; n <= 5; ++n) {
            const int64_t N = 1 << n, E = 2 * N * N;
            double *A = malloc(E * sizeof(double)), *c = malloc(E * sizeof(double)), *B = malloc(E * sizeof(double));
            int64_t *Ai = malloc(E * sizeof(int64_t)), *ci = malloc(E * sizeof(int64_t));
            for (int64_t i = 0; i < E; ++i) {
                s ^= s << 13; s ^= s >> 7; s ^= s << 17;
                Ai[i] = (int64_t)(s % 17) - 8;
                A[i] = (double)Ai[i];
            }
            for (int t = 1; t <= 3; ++t) {
                if (oracle_decompose_f64(n, A, c, t)) return 1;
                if (oracle_decompose_i64(n, Ai, ci, t)) return 2;
                for (int64_t i = 0; i < E; ++i)
                    if (c[i] * (double)N != (double)ci[i]) return 3;
            }
            if (oracle_reconstruct_f64(n, c, B)) return 4;
            for (int64_t i = 0; i < E; ++i)
                if (fabs(B[i] - A[i]) > 1e-12) return 5;
            uint32_t xs[3] = {0, (uint32_t)(N - 1), (uint32_t)(N / 2)}, zs[3] = {(uint32_t)(N - 1), 0, 1};
            double sc[6];
            if (oracle_coeffs_f64(n, A, 3, xs, zs, sc, 2)) return 6;
            for (int i = 0; i < 3; ++i)
                if (sc[2 * i] != c[2 * (xs[i] * N + zs[i])] || sc[2 * i + 1] != c[2 * (xs[i] * N + zs[i]) + 1]) return 7;
            double *rows = malloc(3 * 2 * N * sizeof(double));
            if (oracle_rows_f64(n, A, 3, xs, rows, 3)) return 8;
            for (int i = 0; i < 3; ++i)
                for (int64_t z = 0; z < 2 * N; ++z)
                    if (rows[i * 2 * N + z] != c[2 * xs[i] * N + z]) return 9;
            if (oracle_decompose_f64(0, A, c, 1) != -1) return 10;
            free(rows); free(A); free(c); free(B); free(Ai); free(ci);
        }
        puts("oracle ok");
        return 0;
    }
""")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def test_host_tree_under_sanitizers(tmp_path):
    drv = tmp_path / "tree_driver.cpp"
    drv.write_text(TREE_DRIVER)
    exe = tmp_path / "tree_asan"
    _run(["g++", "-std=c++17", "-pthread", *SAN, "-I", os.path.join(ROOT, "include"),
          os.path.join(ROOT, "paper_2403_11644_amd", "csrc", "host_tree.cpp"), str(drv), "-o", str(exe)])
    r = _run([str(exe)], env=_env())
    assert "tree ok" in r.stdout


def test_oracle_under_sanitizers(tmp_path):
    drv = tmp_path / "oracle_driver.c"
    drv.write_text(ORACLE_DRIVER)
    exe = tmp_path / "oracle_asan"
    _run(["gcc", "-std=c11", "-pthread", *SAN, os.path.join(ROOT, "oracle", "oracle.c"), str(drv), "-lm",
          "-o", str(exe)])
    r = _run([str(exe)], env=_env())
    assert "oracle ok" in r.stdout
