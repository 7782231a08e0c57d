"""hgks_step_static, the step entry point that allocates no device memory (its
workspace is the library's static device array), against hgks_init +
hgks_step on a caller-allocated workspace: calls in a row on boxes of
decreasing size and different workspace layouts (Taylor-Green 32^3; a stretched
channel with walls and constant bulk momentum; an isotropic mode-Z box in the
FP32-flux form), each bitwise equal to the allocating path, with the same time
steps."""
import sys

import numpy as np
import pytest
import torch

from paper_2005_08736_amd import cases, hgks

pytestmark = pytest.mark.gpu


def _runs():
    yield "Taylor-Green 32^3 FP64, 3 steps", cases.tgv_params(32), cases.tgv_state(32), 3
    pc = cases.channel_params(16, 12, 8, body_force_x=0.0, bulk_momentum=1.0)
    yield "channel 16x12x8 bulk momentum, 2 steps", pc, cases.channel_state(pc, seed=4), 2
    pz = dict(cases.isotropic_params(16, 0.5), precision=hgks.PREC_F32FLUX)
    yield "isotropic 16^3 mode Z FP32 form, 2 steps", pz, cases.isotropic_state(16, 0, 0.5), 2


def test_static_workspace_step_matches_the_allocating_step():
    dev = torch.device("cuda:0")
    for name, p, q, n in _runs():
        print(f"[gpu-case] hgks_step_static {name}", flush=True)
        sys.stdout.flush()
        assert hgks.workspace_bytes(p) <= hgks.STATIC_WORKSPACE_BYTES
        a = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
        dts_a = hgks.Solver(p, a).step(n, return_dt=True)
        b = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
        dts_b = hgks.step_static(p, b, n, return_dt=True)
        torch.cuda.synchronize()
        assert dts_a == dts_b, (name, dts_a, dts_b)
        assert torch.equal(a, b), (name, float((a - b).abs().max()))


def test_static_workspace_rejects_a_box_beyond_its_limit():
    p = cases.tgv_params(64)
    assert hgks.workspace_bytes(p) > hgks.STATIC_WORKSPACE_BYTES
    q = torch.zeros((5, 64, 64, 64), dtype=torch.float64, device="cuda:0")
    with pytest.raises(hgks.HgksError) as e:
        hgks.step_static(p, q, 1)
    assert e.value.status == hgks.HGKS_E_WORKSPACE
