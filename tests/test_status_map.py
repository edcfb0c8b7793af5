"""Host-side unit test of the mapping from the error bits that kernels latch
in the device control block to the status a call reports.  The mapping is
plain C++ (csrc/bqs_status_map.h); it is compiled here with g++ and run for
every combination of the four bits."""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <cstdio>
#include "bqs_status_map.h"
int main() {
    for (unsigned e = 0; e < 16; ++e) std::printf("%u %d\n", e, (int)bqs::status_of_device_error(e));
    std::printf("bits %u %u %u %u\n", bqs::ERR_OVERFLOW, bqs::ERR_OFFSETS, bqs::ERR_STALL, bqs::ERR_NAN);
    return 0;
}
"""


def test_device_error_bits_map_to_statuses(tmp_path):
    src = tmp_path / "m.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "m"
    subprocess.run(["g++", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1604_06697_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True)
    lines = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {int(a): int(b) for a, b in (ln.split() for ln in lines if ln and not ln.startswith("bits"))}
    bits = [int(x) for x in next(ln for ln in lines if ln.startswith("bits")).split()[1:]]
    overflow, offsets, stall, nan = bits
    OK, EINVAL, EHIP, ENAN, EOVERFLOW = 0, 1, 4, 5, 6
    assert got[0] == OK
    for e in range(1, 16):
        if e & offsets:
            want = EINVAL      # malformed offsets stop every kernel: reported as a bad argument
        elif e & nan:
            want = ENAN        # the NaN check
        elif e & stall:
            want = EHIP        # a bounded device wait gave up: not an overflow
        else:
            want = EOVERFLOW
        assert got[e] == want, (e, got[e], want)
    assert got[overflow] == EOVERFLOW and got[stall] == EHIP and got[stall | overflow] == EHIP
