"""The header is plain C: a C99 program that includes include/lbm.h (with
-Wall -Wextra -Werror -pedantic) links against the library and calls its
host-side entry points; its results agree with the oracle's EOS."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2205_09186_amd")

PROGRAM = r"""
#include <stdio.h>
#include "lbm.h"

int main(void)
{
    lbm_params p = {0};
    double Tc, rc, pc, g, l;
    p.lattice = LBM_D3Q19;
    p.nx = 64; p.ny = 48; p.nz = 40;
    p.tau = 1.0; p.Tr = 0.8; p.k = 0.1; p.kappa = 0.004;
    p.scheme = LBM_CD6;
    p.collision = LBM_SRT;
    if (lbm_critical(&p, &Tc, &rc, &pc) != LBM_OK) return 2;
    if (lbm_coexistence(&p, &g, &l) != LBM_OK) return 3;
    printf("%zu %.17g %.17g %.17g %.17g %.17g\n", lbm_workspace_bytes(&p), Tc, rc, pc, g, l);
    p.tau = 0.4;                                   /* invalid: tau <= 1/2 */
    {
        double rho0 = 3.0;
        lbm_ctx* c = NULL;
        const int rc_init = lbm_init(&p, &rho0, 0, NULL, 0, NULL, &c);   /* refused before any device work */
        printf("%zu %d %s %s\n", lbm_workspace_bytes(&p), rc_init, c ? "ctx" : "null",
               lbm_last_error(NULL)[0] ? "msg" : "none");
    }
    return 0;
}
"""


def test_header_compiles_as_c_and_links(tmp_path, orc):
    lib = os.path.join(PKG, "liblbm.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    src = tmp_path / "use_lbm.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "use_lbm"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    str(src), "-L", PKG, "-llbm", "-Wl,-rpath," + PKG, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    ws, Tc, rc, pc, g, l = out[0].split()
    assert int(ws) > 19 * 2 * 8 * 64 * 48 * 40
    Tc_o, rc_o, pc_o = orc.pr_critical()
    assert float(Tc) == pytest.approx(Tc_o, rel=1e-12)
    assert float(rc) == pytest.approx(rc_o, rel=1e-12)
    assert float(pc) == pytest.approx(pc_o, rel=1e-12)
    g_o, l_o = orc.maxwell(0.8)
    assert float(g) == pytest.approx(g_o, rel=1e-10) and float(l) == pytest.approx(l_o, rel=1e-10)
    assert out[1].split() == ["0", "-1", "null", "msg"]
