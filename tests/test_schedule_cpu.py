"""The replay schedule the kernels decode (one work item, launch by launch),
checked on the host: every forward step once and in order; then the adjoint
levels of the last segment; then, per earlier segment from the last to the
first, its K recompute steps from its checkpoint followed by its adjoint
levels; every adjoint level T..1 exactly once, in decreasing order; launch
counts as the host plan computes them."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def dump():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "schedule_dump")
    cmd = [HIPCC, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_2603_04070_amd", "csrc"),
           "-o", exe, os.path.join(ROOT, "tests", "capi", "schedule_dump.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]

    def run(T, K, S, Sa):
        out = subprocess.run([exe, str(T), str(K), str(S), str(Sa)], capture_output=True, text=True, check=True).stdout
        return [tuple(int(v) for v in l.split()) for l in out.splitlines()]
    return run


CASES = [(T, K, S, Sa) for S, Sa in ((1, 1), (2, 2), (3, 2)) for T, K in
         [(1, 1), (2, 2), (3, 3), (5, 2), (7, 3), (10, 4), (11, 4), (64, 8), (65, 8), (100, 14), (101, 14),
          (120, 120), (37, 36), (4000, 90), (3407, 82), (100, 12), (4000, 84)]]


@pytest.mark.parametrize("T,K,S,Sa", CASES)
def test_schedule(dump, T, K, S, Sa):
    K = min(K, T)
    J = (T + K - 1) // K
    last = T - (J - 1) * K
    seq = dump(T, K, S, Sa)
    # launch count of the host plan
    steps = -(-T // S) + -(-last // Sa) + (-(-K // S) + -(-K // Sa)) * (J - 1)
    assert len(seq) == steps
    i = 0
    # forward: steps 0..T-1 in order, runs of S
    n = 0
    while n < T:
        ph, n0, j, c = seq[i]
        assert (ph, n0) == (1, n) and 1 <= c <= S and j == n // K
        n += c
        i += 1
    assert n == T

    def adjoint(top, bottom):
        """levels top..bottom (lam^{t-1}..lam^{t-c} for an entry (t, c))"""
        nonlocal i
        lev = top
        while lev >= bottom:
            ph, t, j, c = seq[i]
            assert ph == 3 and t == lev + 1 and 1 <= c <= Sa and lev - c + 1 >= bottom
            lev -= c
            i += 1
        assert lev == bottom - 1

    adjoint(T, (J - 1) * K + 1)
    for j in range(J - 2, -1, -1):
        n = j * K
        while n < (j + 1) * K:
            ph, n0, jj, c = seq[i]
            assert (ph, n0, jj) == (2, n, j) and 1 <= c <= S and n0 + c <= (j + 1) * K
            n += c
            i += 1
        adjoint((j + 1) * K, j * K + 1)
    assert i == len(seq)
