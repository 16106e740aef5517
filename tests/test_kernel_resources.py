"""The hop kernels keep their working set in registers: no spills, no scratch,
and no LDS beyond the buffer in which the wave groups of a work item add their
partial sums (a private array moved to LDS or scratch costs a factor of two in
hop bandwidth).  Checked from the compiler's gfx950 resource report; runs on the
CPU."""
import concurrent.futures
import os
import re
import shutil

import pytest

from paper_1401_2039_amd import build

pytestmark = pytest.mark.skipif(not os.path.exists(build.HIPCC) and shutil.which("hipcc") is None,
                                reason="hipcc not available")

SOURCES = ["api.hip", "solver_kernels.hip"]
WAVE = 64


def combine_lds(S, T, NR):
    """Bytes of the wave-combine buffer: (4/T items) x (T-1 groups) x NR fields x
    24 reals x 64 lanes (FP64 storage computes in double, the others in float)."""
    if T == 1:
        return 0
    real = 8 if S == 0 else 4
    return (4 // T) * (T - 1) * NR * 24 * WAVE * real


def expected_lds(name):
    m = re.search(r"k_hop(?:_sys)?ILi(\d)ELi\d+ELb\dELi\dELi(\d)ELi(\d)ELb\dE", name)
    if m:
        S, T, NR = map(int, m.groups())
        return combine_lds(S, T, NR)
    if re.search(r"k_hop_(sum|upd|res)", name):
        return combine_lds(0, 4, 1)
    return None


@pytest.fixture(scope="module")
def reports():
    with concurrent.futures.ThreadPoolExecutor(len(SOURCES)) as ex:
        out = ex.map(lambda s: build.kernel_resources(os.path.join(build.CSRC, s)), SOURCES)
        return dict(zip(SOURCES, out))


@pytest.mark.parametrize("src", SOURCES)
def test_hop_kernels_do_not_spill(src, reports):
    hops = [(r, expected_lds(r["name"])) for r in reports[src]]
    hops = [(r, e) for r, e in hops if e is not None]
    assert len(hops) >= 8, "hop kernels missing from the resource report"
    bad = [(r["name"][:60], r.get("ScratchSize [bytes/lane]"), r.get("LDS Size [bytes/block]"), e)
           for r, e in hops
           if r.get("ScratchSize [bytes/lane]") != "0" or r.get("VGPRs Spill") != "0"
           or int(r.get("LDS Size [bytes/block]", "-1")) != e]
    assert not bad, f"{len(bad)} hop kernels use scratch or unexpected LDS: {bad[:4]}"
