"""Host-only checks of the C ABI: the library loads, exports what include/asm.h declares,
and rejects malformed requests before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "asm.h")
LIB = os.path.join(ROOT, "paper_1912_01379_amd", "libasm.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(asm_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["asm_plan_create", "asm_plan_run", "asm_plan_vjp", "asm_plan_destroy",
              "asm_last_error", "asm_tn_draw", "asm_uniforms"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build with python -m paper_1912_01379_amd.build"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib.asm_version.restype = ctypes.c_int
    assert lib.asm_version() >= 100


def test_binding_exposes_the_same_names():
    import paper_1912_01379_amd as pk
    assert sorted(pk.EXPORTED) == declared_functions()


def _opts(pk, **kw):
    base = dict(chains=4, burnin=0, sweeps=10, seed=1, precision=pk.ASM_FP32, refresh_every=64,
                want_vjp=0, groups=4, lanes_per_chain=0, use_graph=0, start=0)
    base.update(kw)
    return pk._Options(**base)


def _create(pk, probs, n, opts):
    handle = ctypes.c_void_p()
    rc = pk.lib().asm_plan_create(probs, n, ctypes.byref(opts), None, ctypes.byref(handle))
    return rc, pk.lib().asm_last_error().decode()


def test_invalid_requests_are_rejected_on_the_host():
    """Validation runs before any HIP call, so these need no GPU."""
    import paper_1912_01379_amd as pk
    bs = np.array([0, 5, 10], np.int64)
    fake = 1  # never dereferenced: validation fails first
    good = pk._Problem(M=4, N=10, K=fake, G=fake, sigma=fake, cov=None, B=2,
                       block_start=bs.ctypes.data, k=None, init=None)
    # no problems
    rc, msg = _create(pk, None, 0, _opts(pk))
    assert rc == pk.ASM_EINVAL and "problem" in msg
    # zero chains
    arr = (pk._Problem * 1)(good)
    rc, msg = _create(pk, arr, 1, _opts(pk, chains=0))
    assert rc == pk.ASM_EINVAL and "chains" in msg
    # bad precision
    rc, msg = _create(pk, arr, 1, _opts(pk, precision=7))
    assert rc == pk.ASM_EINVAL
    # partition not ending at N
    bad = np.array([0, 5, 9], np.int64)
    p = pk._Problem(M=4, N=10, K=fake, G=fake, sigma=fake, cov=None, B=2, block_start=bad.ctypes.data,
                    k=None, init=None)
    rc, msg = _create(pk, (pk._Problem * 1)(p), 1, _opts(pk))
    assert rc == pk.ASM_EINVAL and "block_start" in msg
    # empty block
    bad = np.array([0, 5, 5, 10], np.int64)
    p = pk._Problem(M=4, N=10, K=fake, G=fake, sigma=fake, cov=None, B=3, block_start=bad.ctypes.data,
                    k=None, init=None)
    rc, msg = _create(pk, (pk._Problem * 1)(p), 1, _opts(pk))
    assert rc == pk.ASM_EINVAL and "non-empty" in msg
    # both sigma and cov
    p = pk._Problem(M=4, N=10, K=fake, G=fake, sigma=fake, cov=fake, B=2, block_start=bs.ctypes.data,
                    k=None, init=None)
    rc, msg = _create(pk, (pk._Problem * 1)(p), 1, _opts(pk))
    assert rc == pk.ASM_EINVAL and "sigma" in msg
    # negative k
    kk = np.array([1, -1], np.int32)
    p = pk._Problem(M=4, N=10, K=fake, G=fake, sigma=fake, cov=None, B=2, block_start=bs.ctypes.data,
                    k=kk.ctypes.data, init=None)
    rc, msg = _create(pk, (pk._Problem * 1)(p), 1, _opts(pk))
    assert rc == pk.ASM_EINVAL and "k" in msg
    # bad lanes
    rc, msg = _create(pk, arr, 1, _opts(pk, lanes_per_chain=3))
    assert rc == pk.ASM_EINVAL and "lanes" in msg
    # too many groups
    rc, msg = _create(pk, arr, 1, _opts(pk, groups=65))
    assert rc == pk.ASM_EINVAL and "groups" in msg
    # unknown start model
    rc, msg = _create(pk, arr, 1, _opts(pk, start=5))
    assert rc == pk.ASM_EINVAL and "start" in msg


def test_null_plan_calls_fail_cleanly():
    import paper_1912_01379_amd as pk
    L = pk.lib()
    assert L.asm_plan_run(None, None, None, None, None) == pk.ASM_EINVAL
    assert L.asm_plan_vjp(None, None, None, None) == pk.ASM_EINVAL
    assert L.asm_plan_vjp_noalloc(None, None, None, None) == pk.ASM_EINVAL
    assert L.asm_plan_group_means(None, None, None, None) == pk.ASM_EINVAL
    assert L.asm_plan_advance(None, 1) == pk.ASM_EINVAL
    assert L.asm_plan_destroy(None) == pk.ASM_OK


def test_invalid_hierarchies_are_rejected_on_the_host():
    import paper_1912_01379_amd as pk
    fake = 1
    st = np.array([0, 10, 0, 5, 10], np.int64)       # two levels: [0, 10] and [0, 5, 10]
    lb = np.array([1, 2], np.int64)

    def make(levels, level_blocks, B, starts):
        return (pk._Problem * 1)(pk._Problem(M=4, N=10, K=fake, G=fake, sigma=fake, cov=None, B=B,
                                             block_start=starts.ctypes.data, k=None, init=None,
                                             levels=levels, level_blocks=level_blocks))
    rc, msg = _create(pk, make(2, None, 3, st), 1, _opts(pk))
    assert rc == pk.ASM_EINVAL and "level_blocks" in msg
    rc, msg = _create(pk, make(2, lb.ctypes.data, 4, st), 1, _opts(pk))
    assert rc == pk.ASM_EINVAL and "sum" in msg
    bad = np.array([0, 10, 0, 5, 9], np.int64)
    rc, msg = _create(pk, make(2, lb.ctypes.data, 3, bad), 1, _opts(pk))
    assert rc == pk.ASM_EINVAL and "level 1" in msg
    rc, msg = _create(pk, make(65, lb.ctypes.data, 3, st), 1, _opts(pk))
    assert rc == pk.ASM_EINVAL and "levels" in msg
    # two roles are refused with a hierarchy (checked after the GPU setup, so not here)


def test_hierarchy_matches_the_oracle():
    """asm_hierarchy (host code of the library) against the oracle's reading of Fig. 2."""
    import oracle
    import paper_1912_01379_amd as pk
    for N in list(range(1, 140)) + [800, 1000, 4097]:
        for mb in (0, 16, 128):
            got = pk.hierarchy(N, mb)
            ref = oracle.hierarchy(N, mb)
            assert len(got) == len(ref), (N, mb)
            for g, r in zip(got, ref):
                assert np.array_equal(g, r), (N, mb, g, r)
    nl, ns = ctypes.c_int64(), ctypes.c_int64()
    assert pk.lib().asm_hierarchy(0, 0, ctypes.byref(nl), ctypes.byref(ns), None, None) == pk.ASM_EINVAL
    assert pk.lib().asm_hierarchy(5, 0, None, ctypes.byref(ns), None, None) == pk.ASM_EINVAL


def test_a_c_program_uses_the_library(tmp_path):
    """The header is plain C99 and the library links into a C program; the host-only entry
    point runs without a GPU."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(r'''
#include <stdio.h>
#include "asm.h"
int main(void) {
    int64_t levels = 0, n_starts = 0, lb[64], st[64];
    if (asm_hierarchy(8, 0, &levels, &n_starts, lb, st) != ASM_OK) return 1;
    printf("%lld %lld", (long long)levels, (long long)n_starts);
    for (int64_t i = 0; i < n_starts; ++i) printf(" %lld", (long long)st[i]);
    printf(" %d\n", asm_version());
    return 0;
}
''')
    exe = tmp_path / "use"
    libdir = os.path.dirname(LIB)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                           "-L", libdir, "-lasm", "-Wl,-rpath," + libdir, "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split()
    # Fig. 2 on 8 points: [0 8], [0 4 8], [0 1 3 5 7 8], [0 1 ... 8]
    assert out[:2] == ["4", "20"]
    assert [int(x) for x in out[2:-1]] == [0, 8, 0, 4, 8, 0, 1, 3, 5, 7, 8] + list(range(9))
