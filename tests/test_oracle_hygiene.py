"""Hygiene of the FP64 oracle itself (CPU only):

* its step does not depend on the number of OpenMP threads: every cell is
  computed from the previous level alone and the reductions are serial
  sums in a fixed order, so one thread and all threads give the same bits
  (a data race would show up as a difference);
* a driver that calls every entry point of oracle.c, built with gcc's
  address and undefined-behaviour sanitizers, runs clean on 2-D and 3-D
  lattices with periodic, wall and symmetry boundaries.
"""
import os
import shutil
import subprocess
import textwrap

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")


def random_state(dim, n, bc, seed):
    """A seeded interface with a random velocity field and its equilibrium
    populations, perturbed so that every moment the collision reads is live."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    shape = (nz, ny, nx)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    h = (ny / 2 if dim == 2 else nz / 2) + 1.5 * np.cos(2 * np.pi * x / nx)
    d = (y if dim == 2 else z) - h
    phi = 0.5 * (1 + np.tanh(2 * d / 4.0))
    u = 0.02 * rng.standard_normal((3,) + shape)
    if dim == 2:
        u[2] = 0
    p = 1e-3 * rng.standard_normal(shape)
    params = {"dim": dim, "n": list(n), "bc": list(bc), "rho_h": 1.0, "rho_l": 0.05,
              "nu_h": 0.02, "nu_l": 0.05, "W": 4.0, "M": 0.1, "sigma": 1e-3,
              "g": [0.0, -1e-5, 0.0] if dim == 2 else [0.0, 0.0, -1e-5]}
    po = oracle.params_from_dict(params)
    f, g = oracle.init(po, phi, u, p)
    f = f * (1 + 1e-3 * rng.standard_normal(f.shape))
    g = g * (1 + 1e-3 * rng.standard_normal(g.shape))
    return po, f, g


@pytest.mark.parametrize("dim,n,bc", [(2, (24, 20, 1), (0, 1, 0)),
                                      (3, (10, 9, 8), (0, 2, 1)),
                                      (3, (8, 8, 12), (1, 0, 0))])
def test_step_and_reduce_do_not_depend_on_thread_count(dim, n, bc):
    po, f, g = random_state(dim, n, bc, seed=11)
    threads = oracle.num_threads()
    try:
        oracle.set_threads(1)
        f1, g1 = oracle.step(po, f, g, 3)
        r1 = oracle.reduce(po, f1, g1)
        oracle.set_threads(max(threads, 4))
        fa, ga = oracle.step(po, f, g, 3)
        ra = oracle.reduce(po, fa, ga)
    finally:
        oracle.set_threads(threads)
    assert np.array_equal(f1, fa) and np.array_equal(g1, ga)
    assert np.array_equal(r1, ra)


DRIVER = textwrap.dedent(r"""
    #include <math.h>
    #include <stdio.h>
    #include <stdlib.h>
    #include "oracle.h"

    static int run(int dim, int nx, int ny, int nz, int bx, int by, int bz, int edf)
    {
        orc_params p = {0};
        p.dim = dim; p.n[0] = nx; p.n[1] = ny; p.n[2] = nz;
        p.bc[0] = bx; p.bc[1] = by; p.bc[2] = bz;
        p.rho_h = 1.0; p.rho_l = 0.05; p.nu_h = 0.02; p.nu_l = 0.05;
        p.W = 4.0; p.M = 0.1; p.sigma = 1e-3; p.g[dim - 1] = -1e-5;
        p.visc_interp = 1; p.collision = 0;
        p.rate_bulk = p.rate3 = p.rate4 = p.rate5 = p.rate6 = 1.0;
        p.cac_edf = edf;
        const int Q = orc_Q(dim);
        const long N = (long)nx * ny * nz;
        double *phi = malloc(sizeof(double) * N), *u = calloc(3 * N, sizeof(double));
        double *ph = calloc(N, sizeof(double)), *rho = malloc(sizeof(double) * N);
        double *f = malloc(sizeof(double) * Q * N), *g = malloc(sizeof(double) * Q * N);
        double *fo = malloc(sizeof(double) * Q * N), *go = malloc(sizeof(double) * Q * N);
        double *grad = malloc(sizeof(double) * 3 * N), *lap = malloc(sizeof(double) * N);
        double *phiu = calloc(3 * N, sizeof(double));
        for (long i = 0; i < N; ++i) {
            const long x = i % nx, y = (i / nx) % ny, z = i / ((long)nx * ny);
            const double h = 0.5 * (dim == 2 ? ny : nz) + 1.5 * cos(6.283185307179586 * x / nx);
            phi[i] = 0.5 * (1.0 + tanh(0.5 * ((dim == 2 ? y : z) - h)));
            u[i] = 0.01 * sin(0.7 * i);
            u[N + i] = 0.01 * cos(0.3 * i);
            if (dim == 3) u[2 * N + i] = 0.005 * sin(0.11 * i);
        }
        int rc = orc_init(&p, phi, u, ph, f, g);
        rc |= orc_gradients(&p, phi, grad, lap);
        for (int s = 0; s < 3; ++s) {
            rc |= orc_step(&p, f, g, fo, go);
            double *t = f; f = fo; fo = t;
            t = g; g = go; go = t;
        }
        rc |= orc_step_hist(&p, f, g, fo, go, phiu, 0);
        rc |= orc_step_hist(&p, fo, go, f, g, phiu, 1);
        long cells[5] = {0, N / 3, N / 2, N - nx, N - 1};
        double fs[5 * 27], gs[5 * 27];
        rc |= orc_step_sampled(&p, f, g, cells, 5, fs, gs);
        rc |= orc_fields(&p, f, g, phi, rho, u, ph);
        double out5[5];
        rc |= orc_reduce(&p, f, g, out5);
        double fc[27], gc[27], diag[ORC_DIAG_SIZE], pu[3] = {0, 0, 0}, puo[3];
        for (int a = 0; a < Q; ++a) { fc[a] = f[(long)a * N + N / 2]; gc[a] = g[(long)a * N + N / 2]; }
        const double gr[3] = {grad[N / 2], grad[N + N / 2], grad[2 * N + N / 2]};
        rc |= orc_collide_cell(&p, fc, gc, phi[N / 2], gr, lap[N / 2], fs, gs, diag, pu, puo);
        double Pi[27], K[27], back[27], h[27];
        const double uc[3] = {0.02, -0.01, dim == 3 ? 0.015 : 0.0};
        orc_central_moments(dim, gc, uc, Pi);
        orc_cumulants_from_central(dim, Pi, K);
        orc_central_from_cumulants(dim, K, back);
        rc |= orc_populations_from_central(dim, back, uc, h);
        printf("dim %d n %d %d %d rc %d mass %.17g\n", dim, nx, ny, nz, rc, out5[0]);
        free(phi); free(u); free(ph); free(rho); free(f); free(g); free(fo); free(go);
        free(grad); free(lap); free(phiu);
        return rc != 0 || !isfinite(out5[0]);
    }

    int main(void)
    {
        int bad = 0;
        orc_set_threads(4);
        bad |= run(2, 20, 16, 1, 0, 1, 0, 0);
        bad |= run(2, 16, 14, 1, 2, 1, 0, 1);
        bad |= run(3, 8, 7, 6, 0, 2, 1, 0);
        bad |= run(3, 6, 6, 8, 1, 1, 1, 1);
        return bad;
    }
""")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", ORACLE_DIR, "-o", str(exe), str(drv),
                           os.path.join(ORACLE_DIR, "oracle.c"), "-lm"])
    env = dict(os.environ)
    # libgomp keeps its thread pool until exit: leaks are not this test's subject
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=240)
    out = res.stdout + res.stderr
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert out.count(" rc 0 ") == 4, out
