"""The oracle built with the address and undefined-behaviour sanitizers (CPU).

A small driver program (C, linked against the oracle source only) runs a 2D
case with phase change in both directions, a 3D case with an inlet and an
outlet, and the adjoint of a 2D case; any out-of-bounds access, use of freed
memory, leak or undefined behaviour makes the sanitized run fail.
"""
import os
import shutil
import subprocess

import pytest

import oracle

DRIVER = r"""
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int dim, nx, ny, nz, q;
    int mechanics, scheme;
    double tau_ns, tau_ad, j0;
    double force[3];
    double c_eq, k_r, v_m, a_m;
    int periodic[3];
    int xwrap_shift_y;
    int inlet_axis;
    double c_in;
    int phase_change;
    int collision;
    int qs;
    int fluid_open;
    double u_in, rho_out;
} orc_params;
typedef struct orc orc;
orc *orc_create(const orc_params *, const uint8_t *, const double *, const double *, const double *);
void orc_destroy(orc *);
void orc_init(orc *, const double *, const double *, const double *);
void orc_step(orc *, int);
void orc_diag(const orc *, double *);
int orc_adjoint(orc *, int, const double *, double *, double *);

static orc_params base(int dim, int nx, int ny, int nz, int q) {
    orc_params p;
    memset(&p, 0, sizeof p);
    p.dim = dim; p.nx = nx; p.ny = ny; p.nz = nz; p.q = q;
    p.tau_ns = 0.8; p.tau_ad = 0.8; p.j0 = 0.3; p.c_eq = 1.0; p.k_r = 0.05;
    p.v_m = 1.0; p.a_m = 1.0; p.periodic[0] = p.periodic[1] = p.periodic[2] = 1;
    p.inlet_axis = -1; p.rho_out = 1.0;
    return p;
}

int main(void) {
    double d[7];
    /* 2D, phase change: a solid block whose interface starts near phi = 0
       (dissolution) and fluid nodes near phi = 1 (precipitation) */
    {
        int nx = 20, ny = 14;
        long N = (long)nx * ny;
        uint8_t *solid = calloc(N, 1);
        double *phi = calloc(N, sizeof(double)), *c = calloc(N, sizeof(double));
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long n = x + (long)nx * y;
                solid[n] = (x >= 6 && x < 12 && y >= 4 && y < 9) || y == 0;
                phi[n] = solid[n] ? 0.01 : (x == 15 && y == 10 ? 0.999 : 0.0);
                c[n] = 0.5 + 0.05 * ((x * 7 + y * 3) % 11);
            }
        orc_params p = base(2, nx, ny, 1, 9);
        p.phase_change = 1;
        p.c_eq = 0.0;
        orc *o = orc_create(&p, solid, NULL, NULL, phi);
        orc_init(o, NULL, NULL, c);
        orc_step(o, 200);
        orc_diag(o, d);
        orc_destroy(o);
        p.c_eq = 2.0;
        o = orc_create(&p, solid, NULL, NULL, phi);
        orc_init(o, NULL, NULL, c);
        orc_step(o, 200);
        orc_diag(o, d);
        orc_destroy(o);
        free(solid); free(phi); free(c);
    }
    /* 3D, inlet and outlet along z, a solid box, D3Q7 solute */
    {
        int n = 8;
        long N = (long)n * n * n;
        uint8_t *solid = calloc(N, 1);
        for (int z = 2; z < 5; z++)
            for (int y = 3; y < 6; y++)
                for (int x = 2; x < 6; x++) solid[x + n * (y + (long)n * z)] = 1;
        orc_params p = base(3, n, n, n, 19);
        p.inlet_axis = 2; p.c_in = 2.0; p.force[2] = 1e-5; p.qs = 7;
        orc *o = orc_create(&p, solid, NULL, NULL, NULL);
        orc_init(o, NULL, NULL, NULL);
        orc_step(o, 50);
        orc_diag(o, d);
        orc_destroy(o);
        free(solid);
    }
    /* adjoint, 2D channel with disks, TRT */
    {
        int nx = 16, ny = 12;
        long N = (long)nx * ny;
        uint8_t *solid = calloc(N, 1);
        double *dl = calloc(N, sizeof(double)), *g = calloc(N, sizeof(double));
        double *lam = calloc(N * 9, sizeof(double));
        for (int x = 0; x < nx; x++) { solid[x] = 1; solid[x + (long)nx * (ny - 1)] = 1; }
        solid[5 + nx * 5] = solid[6 + nx * 5] = solid[5 + nx * 6] = 1;
        for (long k = 0; k < N; k++) dl[k] = solid[k] ? 0.0 : 0.01 * (k % 7);
        orc_params p = base(2, nx, ny, 1, 9);
        p.collision = 1; p.v_m = 0.0;
        orc *o = orc_create(&p, solid, NULL, NULL, NULL);
        orc_init(o, NULL, NULL, NULL);
        if (orc_adjoint(o, 30, dl, g, lam) != 0) return 3;
        orc_destroy(o);
        free(solid); free(dl); free(g); free(lam);
    }
    return 0;
}
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", str(exe), str(drv),
           oracle.SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
