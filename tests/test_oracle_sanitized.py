"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a small driver runs the start-up, 20 steps in 1/2/3-D with
expansion, negative masses and a vacuum term, and the random-field
routines; any out-of-bounds access, leak or undefined operation fails it."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")

DRIVER = r'''
#include "oracle.c"
#include "grf.c"
#include <stdio.h>

int main(void)
{
    double rho_sum = 0.0;
    for (int dims = 1; dims <= 3; dims++) {
        or_params p;
        memset(&p, 0, sizeof(p));
        p.dims = dims;
        p.N = dims == 3 ? 8 : (dims == 2 ? 16 : 32);
        p.nfields = 3;
        p.expansion = dims != 2;
        p.L = 4.0;
        p.dt = 0.01;
        p.lambda = 1.0;
        p.G[1] = 50.0;
        p.G[2] = 20.0;
        p.mu2[0] = -1.0;
        p.mu2[2] = 0.3;
        p.kappa = 0.05;
        p.vacuum = 0.25;
        int64_t ns = 1;
        for (int d = 0; d < dims; d++) ns *= p.N;
        double *phi = malloc(sizeof(double) * 3 * ns), *phid = malloc(sizeof(double) * 3 * ns);
        double *f = malloc(sizeof(double) * 3 * ns), *pi = malloc(sizeof(double) * 3 * ns);
        for (int64_t k = 0; k < 3 * ns; k++) {
            phi[k] = 0.1 * sin(0.37 * (double)k);
            phid[k] = 0.05 * cos(0.11 * (double)k);
        }
        or_state st, log[20];
        or_start(&p, phi, phid, f, pi, &st);
        or_run(&p, f, pi, &st, 20, log);
        rho_sum += st.rho;

        const int W = 2 * (p.N / 4) + 1;
        int64_t box = 1;
        for (int d = 0; d < dims; d++) box *= W;
        double *re = malloc(sizeof(double) * box), *im = malloc(sizeof(double) * box);
        or_grf_modes(7, 1, 0, dims, p.N, p.L, 1e-3, 3.0, re, im);
        int64_t sites[3] = {0, ns / 2, ns - 1};
        double out[3];
        or_grf_sites(dims, p.N, re, im, 3, sites, out);
        rho_sum += out[0] * 0.0;
        free(re); free(im); free(phi); free(phid); free(f); free(pi);
    }
    printf("done %.6e\n", rho_sum);
    return 0;
}
'''


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_sanitizers(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.check_call(["gcc", "-std=gnu99", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-I", ORACLE, "-o", str(exe), str(src), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    assert r.stdout.startswith("done")
