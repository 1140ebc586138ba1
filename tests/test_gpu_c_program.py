"""The library from a plain C program, no Python or PyTorch in the process:
hipMalloc for the workspace, lbm_init / lbm_step / lbm_macros /
lbm_spurious_max / lbm_free on the null stream, on a D2Q9 CD4 droplet and a
D3Q19 CD6 droplet; the fields match the oracle to 1e-11."""
import os
import subprocess

import numpy as np
import pytest

from paper_2205_09186_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2205_09186_amd")

PROGRAM = r"""
#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include "lbm.h"

/* usage: prog lattice nx ny nz scheme Tr k kappa steps rho0.bin out.bin */
int main(int argc, char** argv)
{
    if (argc != 12) return 2;
    lbm_params p = {0};
    p.lattice = atoi(argv[1]); p.nx = atoi(argv[2]); p.ny = atoi(argv[3]); p.nz = atoi(argv[4]);
    p.scheme = atoi(argv[5]); p.Tr = atof(argv[6]); p.k = atof(argv[7]); p.kappa = atof(argv[8]);
    p.tau = 1.0;
    const long steps = atol(argv[9]);
    const size_t n = (size_t)p.nx * p.ny * p.nz;
    double* rho0 = malloc(n * sizeof(double));
    double* out = malloc(4 * n * sizeof(double));
    FILE* f = fopen(argv[10], "rb");
    if (!f || fread(rho0, sizeof(double), n, f) != n) return 3;
    fclose(f);
    const size_t ws = lbm_workspace_bytes(&p);
    void* d_ws = NULL;
    if (ws == 0 || hipMalloc(&d_ws, ws) != hipSuccess) return 4;
    lbm_ctx* c = NULL;
    int rc = lbm_init(&p, rho0, 0, d_ws, ws, NULL, &c);
    if (rc != LBM_OK) { fprintf(stderr, "init: %s\n", lbm_last_error(NULL)); return 5; }
    rc = lbm_step(c, steps);
    if (rc == LBM_OK) rc = lbm_macros(c, out, out + n, out + 2 * n, p.lattice == LBM_D3Q19 ? out + 3 * n : NULL, 0);
    double U = 0.0, M = 0.0;
    if (rc == LBM_OK) rc = lbm_spurious_max(c, &U, &M);
    if (rc != LBM_OK) { fprintf(stderr, "run: %s\n", lbm_last_error(c)); return 6; }
    printf("%ld %.17g %.17g\n", lbm_steps_done(c), U, M);
    lbm_free(c);
    hipFree(d_ws);
    f = fopen(argv[11], "wb");
    if (!f || fwrite(out, sizeof(double), 4 * n, f) != 4 * n) return 7;
    fclose(f);
    free(rho0);
    free(out);
    return 0;
}
"""


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    d = tmp_path_factory.mktemp("cprog")
    src = d / "run_lbm.c"
    src.write_text(PROGRAM)
    exe = d / "run_lbm"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-L", PKG, "-llbm", "-Wl,-rpath," + PKG,
                    "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)], check=True)
    return exe, d


@pytest.mark.parametrize("lat,shape,scheme,steps", [(0, (40, 44), "CD4", 60), (1, (12, 14, 16), "CD6", 12)])
def test_c_program_against_oracle(prog, orc, lat, shape, scheme, steps):
    exe, d = prog
    g, l = orc.maxwell(0.8)
    rho0 = inputs.droplet(shape, min(shape) / 4, 4.0, g, l)
    nz, ny, nx = ((1,) + shape) if lat == 0 else shape
    (d / "rho0.bin").write_bytes(np.ascontiguousarray(rho0, np.float64).tobytes())
    sch = orc.SCHEME_NAMES[scheme]
    print(f"case C program lattice={lat} shape={shape} scheme={scheme} steps={steps}", flush=True)
    r = subprocess.run([str(exe), str(lat), str(nx), str(ny), str(nz), str(sch), "0.8", "0.16", "0.004", str(steps),
                        str(d / "rho0.bin"), str(d / "out.bin")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    done, U, M = r.stdout.split()
    assert int(done) == steps
    out = np.fromfile(d / "out.bin", dtype=np.float64).reshape(4, -1)
    o = orc.Sim(orc.Params(lattice=lat, nx=nx, ny=ny, nz=nz, Tr=0.8, k=0.16, kappa=0.004, scheme=sch), rho0)
    o.step(steps)
    ro, vxo, vyo, vzo = (a.reshape(-1) for a in o.macros())
    err = max(np.abs(out[0] - ro).max(), np.abs(out[1] - vxo).max(), np.abs(out[2] - vyo).max())
    if lat == 1:
        err = max(err, np.abs(out[3] - vzo).max())
    assert err <= 1e-11, err
    Uo, Mo = o.observables()
    assert float(U) == pytest.approx(Uo, abs=1e-11) and float(M) == pytest.approx(Mo, rel=1e-13)
