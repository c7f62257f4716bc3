"""The C ABI without a GPU: the header compiles as C, the library loads and
exports every declared function, and its host-only logic (Philox block,
sample-size draws of Algorithm 1) agrees bit for bit with the oracle."""

import ctypes as ct
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from oracle import bigmeans as obm
from oracle import rng as orng
from tests.conftest import ROOT, gpu_available

HEADER = os.path.join(ROOT, "include", "bigmeans.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"BM_API\s+[\w\s\*]+?\b(bm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2403_18766_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2403_18766_amd import build
        build.build()
    return _lib.load()


def test_header_compiles_as_c(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "t.c"
    src.write_text('#include "bigmeans.h"\nint main(void){bm_params p; (void)p; return bm_version();}\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-fsyntax-only",
                        "-I", os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_c_program_links_and_calls_the_library(lib, tmp_path):
    # a C program built against the header and linked with libbigmeans.so
    # calls the host-only entry points; its output must match the oracle
    from paper_2403_18766_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "prog.c"
    src.write_text(r"""
#include <inttypes.h>
#include <stdio.h>
#include "bigmeans.h"
int main(void) {
  uint64_t ctr[4] = {3, 1, 4, 1}, key[2] = {5, 9}, out[4];
  bm_philox4x64(ctr, key, out);
  printf("%d\n", bm_version());
  printf("%" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 "\n", out[0], out[1], out[2], out[3]);
  bm_params p = {0};
  p.m = 1000000; p.s_min = 4096; p.s_max = 65536; p.n = 28; p.k = 25; p.workers = 32;
  p.size_policy = BM_SIZE_LOGUNIFORM; p.seed = 0;
  for (int t = 0; t < 3; ++t) {
    int64_t s; int32_t b;
    if (bm_draw_size(&p, 7, t, NULL, NULL, 0, 0, &s, &b) != BM_OK) return 2;
    printf("%" PRId64 "\n", s);
  }
  p.s_min = 0;
  int64_t s; int32_t b;
  return bm_draw_size(&p, 7, 0, NULL, NULL, 0, 0, &s, &b) == BM_E_ARG ? 0 : 3;
}
""")
    exe = tmp_path / "prog"
    libdir = os.path.dirname(_lib.LIB_PATH)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                        str(src), "-o", str(exe), "-L", libdir, "-lbigmeans",
                        "-Wl,-rpath," + libdir], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stderr)
    lines = r.stdout.split()
    assert int(lines[0]) == 2
    assert tuple(int(v) for v in lines[1:5]) == orng.philox_block_scalar((3, 1, 4, 1), (5, 9))
    P = obm.Params(k=25, workers=32, rounds_T=3, s_min=4096, s_max=65536,
                   size_policy=obm.SIZE_LOGUNIFORM, seed=0)
    assert [int(v) for v in lines[5:8]] == [obm.draw_size(P, 7, t, None)[0] for t in range(3)]


def test_every_declared_symbol_is_exported(lib):
    from paper_2403_18766_amd import _lib
    declared = _declared_functions()
    assert len(declared) >= 12
    bound = {name for name, _, _ in _lib.SIGNATURES}
    assert set(declared) == bound
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.bm_version() == 2


def test_struct_layout_matches_header(lib):
    from paper_2403_18766_amd import _lib
    assert ct.sizeof(_lib.Params) == 80
    assert _lib.Params.tol.offset == 64 and _lib.Params.seed.offset == 72
    assert ct.sizeof(_lib.Result) == 72


def test_philox_block_matches_oracle(lib):
    from paper_2403_18766_amd import api
    r = np.random.default_rng(0)
    for _ in range(300):
        ctr = tuple(int(v) for v in r.integers(0, 2**64, size=4, dtype=np.uint64))
        key = tuple(int(v) for v in r.integers(0, 2**64, size=2, dtype=np.uint64))
        assert api.philox4x64(ctr, key) == orng.philox_block_scalar(ctr, key)


@pytest.mark.parametrize("policy", [obm.SIZE_UNIFORM, obm.SIZE_FIXED, obm.SIZE_LOGUNIFORM,
                                    obm.SIZE_BINS, obm.SIZE_SHRINK])
def test_size_draws_match_oracle(lib, policy):
    from paper_2403_18766_amd import api
    rr = np.random.default_rng(policy)
    for (a, b) in [(1000, 4000), (4096, 65536), (4096, 131072), (7, 7), (1, 2)]:
        if policy == obm.SIZE_FIXED:
            b = a
        op = obm.Params(k=1, workers=1, rounds_T=1, s_min=a, s_max=b, size_policy=policy, seed=42)
        gp = api.RunParams(k=1, workers=1, rounds_T=1, s_min=a, s_max=b, size_policy=policy,
                           seed=42)
        for t in range(0, 60):
            acc = [int(v) for v in rr.integers(0, 20, size=5)]
            passes = [x + int(v) for x, v in zip(acc, rr.integers(0, 20, size=5))]
            stats = {"acc": acc, "passes": passes}
            cnt = int(rr.integers(0, 6))
            lsum = int(sum(rr.integers(a, b + 1, size=cnt))) if cnt else 0
            for w in (0, 1, 7, 63):
                want = obm.draw_size(op, w, t, stats, (lsum, cnt))
                got = api.draw_size(gp, 10**7, 4, w, t, acc, passes, lsum, cnt)
                assert got == want, (a, b, t, w)


def test_draw_size_rejects_bad_arguments(lib):
    from paper_2403_18766_amd import _lib
    p = _lib.Params(m=100, s_min=50, s_max=10, n=2, k=2, workers=1, rounds_T=1, passes_p=1,
                    max_iter=1, n_candidates=1, size_policy=0, prec=0, batched=1, tol=0.0, seed=0)
    s = ct.c_int64()
    b = ct.c_int32()
    assert lib.bm_draw_size(ct.byref(p), 0, 0, None, None, 0, 0, ct.byref(s), ct.byref(b)) == _lib.BM_E_ARG
    p.s_max = 100
    p.size_policy = 5
    assert lib.bm_draw_size(ct.byref(p), 0, 0, None, None, 0, 0, ct.byref(s), ct.byref(b)) == _lib.BM_E_ARG
    p.size_policy = 4
    assert lib.bm_draw_size(ct.byref(p), 0, 1, None, None, 10, -1, ct.byref(s), ct.byref(b)) == _lib.BM_E_ARG


def test_create_without_gpu_reports_state_error(lib):
    if gpu_available():
        pytest.skip("a GPU is present")
    from paper_2403_18766_amd import _lib
    out = ct.c_void_p()
    assert lib.bm_create(0, None, ct.byref(out)) == _lib.BM_E_STATE
    assert out.value is None
    lib.bm_destroy(None)                       # NULL is ignored


def test_binding_refuses_cpu_tensors(lib):
    import torch
    from paper_2403_18766_amd import api
    X = torch.zeros((10, 2))
    with pytest.raises(ValueError):
        api.objective(X, X[:2])
