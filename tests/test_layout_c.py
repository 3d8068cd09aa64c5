"""Struct sizes of include/morse.h as a C compiler lays them out (host gcc)."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_struct_sizes():
    src = r"""
#include <stdio.h>
#include "morse.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(morse_grid2d), sizeof(morse_map_view),
         sizeof(morse_lightcurves), sizeof(morse_trajectories), sizeof(morse_search_out),
         sizeof(morse_lbfgs_opts), sizeof(morse_map_stats));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    assert list(map(int, out)) == [40, 48, 48, 72, 64, 32, 48]
