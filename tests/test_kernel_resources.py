"""The hop kernels keep their whole working set in registers: no spills to
scratch and no private arrays moved to LDS (either costs a factor of two in
hop bandwidth).  Checked from the compiler's gfx950 resource report; runs on
the CPU."""
import concurrent.futures
import os
import shutil

import pytest

from paper_1401_2039_amd import build

HOP_KERNELS = ("k_hop", "k_hop_sys", "k_hop_sum", "k_hop_upd", "k_hop_res")

pytestmark = pytest.mark.skipif(not os.path.exists(build.HIPCC) and shutil.which("hipcc") is None,
                                reason="hipcc not available")


def _is_hop(name):
    return any(f"{len(k)}{k}I" in name for k in HOP_KERNELS)


SOURCES = ["api.hip", "solver_kernels.hip"]


@pytest.fixture(scope="module")
def reports():
    with concurrent.futures.ThreadPoolExecutor(len(SOURCES)) as ex:
        out = ex.map(lambda s: build.kernel_resources(os.path.join(build.CSRC, s)), SOURCES)
        return dict(zip(SOURCES, out))


@pytest.mark.parametrize("src", SOURCES)
def test_hop_kernels_do_not_spill(src, reports):
    rows = reports[src]
    hops = [r for r in rows if _is_hop(r["name"])]
    assert hops, "no hop kernels found in the resource report"
    bad = [(r["name"], r.get("ScratchSize [bytes/lane]"), r.get("LDS Size [bytes/block]"), r.get("VGPRs Spill"))
           for r in hops
           if r.get("ScratchSize [bytes/lane]") != "0" or r.get("LDS Size [bytes/block]") != "0"
           or r.get("VGPRs Spill") != "0"]
    assert not bad, f"{len(bad)} hop kernels use scratch or LDS: {bad[:4]}"
