"""The boundary is a C ABI: include/hmps.h must compile as strict C99 (and
as C++, through its extern "C" guard), and a C program must link against
libhmps.so and call the entry points that need no GPU: hmps_gate (checked
against the closed form of its trace), hmps_workspace_bytes, hmps_schedule
on a two-site chain, hmps_create's argument checks (including the
declared but unbuilt split-bf16 precision) and hmps_last_error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1910_09142_amd")

PROGRAM = r"""
#include <math.h>
#include <stdio.h>
#include <string.h>
#include "hmps.h"

static int fails = 0;
#define CHECK(c) do { if (!(c)) { printf("FAIL %s\n", #c); ++fails; } } while (0)

int main(void) {
  double g[81];
  double tr = 0.0, x = 0.1, J = 1.0;
  int i;
  CHECK(hmps_gate(J, x, g) == HMPS_OK);
  /* trace of exp(-x J S.S) over the spin sectors S = 0, 1, 2 */
  for (i = 0; i < 9; ++i) tr += g[10 * i];
  CHECK(fabs(tr - (exp(2 * x) + 3 * exp(x) + 5 * exp(-x))) < 1e-13);
  CHECK(hmps_gate(J, x, NULL) == HMPS_E_INVALID);
  CHECK(hmps_workspace_bytes(1, 8, 32, 7) > 0);
  CHECK(hmps_workspace_bytes(2, 8, 32, 7) > hmps_workspace_bytes(1, 8, 32, 7));
  {
    int32_t bi[1] = {0}, bj[1] = {1}, order[2] = {0, 1};
    double Jb[1] = {1.0};
    uint8_t cl[2] = {0, 0};
    hmps_lattice lat;
    int32_t n_sites = 0, n_updates = 0;
    memset(&lat, 0, sizeof lat);
    lat.n_phys = 2;
    lat.n_bonds = 1;
    lat.bond_i = bi;
    lat.bond_j = bj;
    lat.bond_J = Jb;
    lat.mps_order = order;
    lat.in_cluster = cl;
    CHECK(hmps_schedule(&lat, &n_sites, &n_updates, NULL, NULL, 0) == HMPS_OK);
    CHECK(n_sites == 2);
    CHECK(n_updates == 2); /* the bond forward, then backward */
  }
  {
    hmps_ctx *ctx = NULL;
    hmps_options opt;
    memset(&opt, 0, sizeof opt);
    CHECK(hmps_create(&ctx, NULL) == HMPS_E_INVALID);
    CHECK(hmps_create(&ctx, &opt) == HMPS_E_INVALID); /* no capacities */
    opt.max_chains = 1;
    opt.max_sites = 8;
    opt.chi_cap = 32;
    opt.max_bonds = 7;
    CHECK(hmps_create(&ctx, &opt) == HMPS_E_NOMEM);   /* no workspace */
    CHECK(ctx == NULL);
    opt.precision = HMPS_PREC_MIXED_BF16X3;           /* declared, not built */
    CHECK(hmps_create(&ctx, &opt) == HMPS_E_INVALID);
    CHECK(ctx == NULL);
    opt.precision = HMPS_PREC_FP64;
    CHECK((HMPS_MEASURE_ENERGY | HMPS_MEASURE_BONDS | HMPS_MEASURE_LOGW |
           HMPS_MEASURE_QN) == HMPS_MEASURE_ALL);
    CHECK(strcmp(hmps_last_error(NULL), "null context") == 0);
    hmps_destroy(NULL);
  }
  printf("%s\n", fails ? "FAILED" : "ok");
  return fails != 0;
}
"""


def build(tmp_path, compiler, std, ext):
    src = tmp_path / f"abi_check.{ext}"
    src.write_text(PROGRAM)
    exe = tmp_path / f"abi_check_{compiler}"
    cmd = [compiler, f"-std={std}", "-Wall", "-Wextra", "-pedantic",
           "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
           "-L", LIB_DIR, "-lhmps", f"-Wl,-rpath,{LIB_DIR}", "-lm",
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("compiler, std, ext", [("gcc", "c99", "c"),
                                                 ("g++", "c++17", "cpp")])
def test_header_compiles_links_and_runs(tmp_path, compiler, std, ext):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    if not os.path.exists(os.path.join(LIB_DIR, "libhmps.so")):
        pytest.fail("libhmps.so is missing: build it first")
    exe = build(tmp_path, compiler, std, ext)
    r = subprocess.run([str(exe)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
