"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host only): a small
driver runs every exported routine on a ragged box (initial state, steps with the general tau
path, pressure tensor, velocity, single-node collision, noise) and must finish without a
sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
double ora_psi(double n, int kind);
void ora_init_density(int nx, int ny, int nz, int geom, int slab_axis, double R, double w,
                      double n_in, double n_out, double noise_amp, uint64_t seed, double* n);
void ora_init_populations(const double* n, int nx, int ny, int nz, double G, int kind, double* f);
void ora_run(double* f, int nx, int ny, int nz, double G, double tau, int kind, long long nsteps);
void ora_pressure_tensor(const double* f, int nx, int ny, int nz, double G, int kind, double* P);
void ora_velocity(const double* f, int nx, int ny, int nz, double G, int kind, double* j, double* u);
void ora_collide_at(const double* f, int nx, int ny, int nz, double G, double tau, int kind, int x,
                    int y, int z, double* out);
double ora_noise(uint64_t seed, uint64_t linear_index, double amp);

int main(void)
{
    const int nx = 7, ny = 5, nz = 6;
    const size_t N = (size_t)nx * ny * nz;
    double* n = malloc(N * sizeof(double));
    double* f = malloc(19 * N * sizeof(double));
    double* P = malloc(6 * N * sizeof(double));
    double* j = malloc(3 * N * sizeof(double));
    double* u = malloc(3 * N * sizeof(double));
    double out[19];
    for (int kind = 0; kind < 2; ++kind) {
        const double G = kind == 0 ? -1.3 * exp(2.0) : -1.3 * 4.0;
        for (int geom = 0; geom < 3; ++geom) {
            ora_init_density(nx, ny, nz, geom, 2, 2.0, 1.0, 2.0, 0.5, 1e-3, 5, n);
            ora_init_populations(n, nx, ny, nz, G, kind, f);
            ora_run(f, nx, ny, nz, G, 0.8, kind, 3);
            ora_pressure_tensor(f, nx, ny, nz, G, kind, P);
            ora_velocity(f, nx, ny, nz, G, kind, j, u);
            ora_collide_at(f, nx, ny, nz, G, 1.0, kind, nx - 1, 0, nz - 1, out);
            for (size_t k = 0; k < 19 * N; ++k)
                if (!isfinite(f[k])) { printf("non-finite\n"); return 1; }
        }
    }
    if (!isfinite(ora_noise(1, 2, 1e-3) + ora_psi(1.0, 0))) return 1;
    free(n); free(f); free(P); free(j); free(u);
    printf("ok\n");
    return 0;
}
'''


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = [gcc, "-g", "-O1", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "oracle", "lbm_oracle.c"), str(drv), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("sanitizers unavailable: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the sanitizer runtime need not be first among the libraries
    # the environment already loads into every process
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip() == "ok"
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
