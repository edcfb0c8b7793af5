"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle: a driver that sorts keys, pairs, segments and records of many
  shapes (including tiny blocks that reach every branch of the final
  partition phase) with the oracle compiled with both sanitizers; any
  out-of-bounds access, use after free, leak or undefined operation ends
  the run with an error.
* The host runtime of the library: bqs_api.hip with its host code compiled
  with both sanitizers (device code unchanged), linked with the kernel
  objects of the regular build, driven through the C ABI on paths that need
  no GPU: contexts, parameters, workspace sizes and argument errors.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]

ORACLE_DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include "bqs_oracle.cpp"

template <class K> static bool sorted(const std::vector<K>& a) {
    for (size_t i = 1; i < a.size(); ++i) if (a[i] < a[i - 1]) return false;
    return true;
}

int main() {
    std::mt19937_64 g(7);
    const int64_t sizes[] = {0, 1, 2, 3, 5, 16, 17, 129, 256, 257, 1000, 4099, 65537};
    const int64_t blocks[] = {0, 1, 2, 3, 4, 7};
    for (int64_t n : sizes) {
        for (int64_t b : blocks) {
            for (int dist = 0; dist < 4; ++dist) {
                std::vector<int32_t> a(n);
                for (int64_t i = 0; i < n; ++i)
                    a[i] = dist == 0 ? int32_t(g()) : dist == 1 ? int32_t(i) : dist == 2 ? int32_t(n - i) : int32_t(g() % 3);
                oracle_params p{};
                p.block = b;
                p.is_thresh = b ? 2 : 0;
                p.depth_limit = -1;
                p.check = 1;
                if (oracle_sort(a.data(), n, OR_I32, &p) != OR_OK || !sorted(a) || p.check_failures) return 1;
            }
        }
        std::vector<double> f(n);
        for (int64_t i = 0; i < n; ++i) f[i] = double(int64_t(g() % 2001) - 1000) / 7.0;
        if (n > 1) f[0] = -0.0;
        oracle_params p{};
        p.depth_limit = -1;
        if (oracle_sort(f.data(), n, OR_F64, &p) != OR_OK) return 2;
        std::vector<uint64_t> k(n);
        std::vector<uint32_t> v(n);
        for (int64_t i = 0; i < n; ++i) { k[i] = g() % 64; v[i] = uint32_t(i); }
        oracle_params q{};
        q.depth_limit = 0;  // heapsort from the start
        if (oracle_sort_pairs(k.data(), v.data(), n, OR_U64, 4, &q) != OR_OK || !sorted(k)) return 3;
        if (oracle_std_sort(k.data(), n, OR_U64) != OR_OK) return 4;
    }
    std::vector<int32_t> s(5000);
    for (auto& x : s) x = int32_t(g());
    const int64_t offs[] = {0, 0, 1, 17, 1000, 1000, 5000};
    oracle_params p{};
    p.depth_limit = -1;
    if (oracle_sort_segments(s.data(), offs, 6, OR_I32, &p) != OR_OK) return 5;
    std::vector<int32_t> rec(21 * 300);
    for (auto& x : rec) x = int32_t(g() % 100);
    if (oracle_sort_records(rec.data(), 300, 2, &p) != OR_OK) return 6;
    std::vector<double> vec(10 * 300);
    for (auto& x : vec) x = double(g() % 1000) / 10.0;
    if (oracle_sort_records(vec.data(), 300, 1, &p) != OR_OK) return 7;
    std::vector<double> nan(4, 0.0);
    nan[2] = std::nan("");
    if (oracle_sort(nan.data(), 4, OR_F64, &p) != OR_ENAN) return 8;
    std::puts("oracle sanitizer run ok");
    return 0;
}
"""


def test_oracle_under_sanitizers(tmp_path):
    src = tmp_path / "drv.cpp"
    src.write_text(ORACLE_DRIVER)
    exe = tmp_path / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", *SAN, "-I", os.path.join(ROOT, "oracle"),
                    str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout


HOST_DRIVER = r"""
#include <cstdio>
#include <initializer_list>
#include "bqs.h"
int main() {
    bqs_ctx* c = nullptr;
    if (bqs_ctx_create(&c) != BQS_OK) return 1;
    for (int p = 0; p < 20; ++p) { bqs_ctx_set_param(c, p, 3); bqs_ctx_get_param(c, p); }
    bqs_ctx_set_param(c, BQS_PARAM_MODE, BQS_MODE_ASYNC);
    bqs_ctx_set_param(c, BQS_PARAM_PIVOT_MODE, 0);
    bqs_ctx_set_param(c, BQS_PARAM_TILE_EPT, 0);
    for (long long n : {0LL, 1LL, 2LL, 1000LL, 1LL << 20, 3000000000LL})
        for (int dt = 0; dt <= 7; ++dt)
            for (int vb : {0, 4, 8, 3})
                for (long long k : {1LL, 7LL, 20000LL}) bqs_workspace_bytes(c, n, (bqs_dtype)dt, vb, k);
    void* fake = reinterpret_cast<void*>(64);
    if (bqs_sort(nullptr, 10, BQS_I32, c) != BQS_EINVAL) return 2;
    if (bqs_sort(fake, 10, (bqs_dtype)42, c) != BQS_EDTYPE) return 3;
    if (bqs_sort(fake, 10, BQS_I32, c) != BQS_EINVAL) return 4;  // no workspace
    if (bqs_sort(fake, 1, BQS_I32, c) != BQS_OK) return 5;
    if (bqs_sort_pairs(fake, fake, 10, BQS_U64, 3, c) != BQS_EDTYPE) return 6;
    if (bqs_sort_segments(fake, nullptr, 3, 10, BQS_I32, c) != BQS_EINVAL) return 7;
    if (bqs_ctx_set_workspace(c, reinterpret_cast<void*>(1 << 20), 1 << 30) != BQS_OK) return 8;
    if (bqs_sort(reinterpret_cast<void*>((1 << 20) + 4096), 1000, BQS_I32, c) != BQS_EINVAL) return 9;
    if (bqs_sort_records(fake, fake, 10, 9, c) != BQS_EDTYPE) return 10;
    if (bqs_sort_noalloc(fake, 1LL << 24, BQS_I32, nullptr, nullptr) != BQS_ETOOBIG) return 11;
    for (int s = 0; s < 9; ++s) bqs_status_str((bqs_status)s);
    bqs_stats st;
    if (bqs_ctx_get_stats(c, &st) != BQS_OK) return 12;
    bqs_ctx_destroy(c);
    bqs_ctx_destroy(nullptr);
    std::puts("host runtime sanitizer run ok");
    return 0;
}
"""


def test_host_runtime_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    objs = [os.path.join(ROOT, "paper_1604_06697_amd", "_build", f + ".o")
            for f in ("bqs_keys", "bqs_pairs32", "bqs_pairs64")]
    if not os.path.exists(hipcc) or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs hipcc and the regular build's kernel objects")
    csrc = os.path.join(ROOT, "paper_1604_06697_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]
    api = tmp_path / "api.o"
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san, *inc,
                    "-c", os.path.join(csrc, "bqs_api.hip"), "-o", str(api)], check=True, capture_output=True)
    drv = tmp_path / "drv.cpp"
    drv.write_text(HOST_DRIVER)
    exe = tmp_path / "drv"
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", *host_san, *inc, "-x", "c++",
                    str(drv), "-x", "none", str(api), *objs, "-o", str(exe)], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_odr_violation=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
