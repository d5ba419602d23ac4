"""Host-side checks of the counting sort's range guards (guards.h): the
predicates its kernels use to skip a scatter that a wrong scan of the slot
counts would send out of range, and the mapping of the preparation flags to
status codes. Compiled for the host with g++ (the header holds no HIP types);
no GPU involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_0711_2023_amd", "csrc")

SRC = r'''
#include <cstdio>
#include "guards.h"
using namespace tk;
int main() {
    int bad = 0;
    // a scan total other than the entry count fails
    bad += !order_total_ok(10, 10);
    bad += order_total_ok(9, 10);
    bad += order_total_ok(11, 10);
    // positions inside the slot's range pass, others fail
    bad += !order_pos_ok(3, 3, 5, 10);
    bad += !order_pos_ok(4, 3, 5, 10);
    bad += order_pos_ok(5, 3, 5, 10);    // one past the slot
    bad += order_pos_ok(2, 3, 5, 10);    // before the slot
    bad += order_pos_ok(9, 8, 11, 10);   // slot end beyond the output
    bad += order_pos_ok(0, -1, 2, 10);   // negative begin
    bad += order_pos_ok(4, 5, 3, 10);    // inverted range
    bad += order_pos_ok(3, 3, 3, 10);    // empty slot
    // flags -> status: index, value, ordering (device), none
    bad += prep_status(0) != 0;
    bad += prep_status(1) != -2;
    bad += prep_status(2) != -3;
    bad += prep_status(3) != -2;
    bad += prep_status(kFlagOrderCheck) != -6;
    bad += prep_status(kFlagOrderCheck | 2) != -3;
    printf("%d\n", bad);
    return bad != 0;
}
'''


def test_order_guards_host(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    src = tmp_path / "guards_test.cpp"
    src.write_text(SRC)
    exe = tmp_path / "guards_test"
    subprocess.run([cxx, "-std=c++17", "-I", HDR, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "0", r.stdout
