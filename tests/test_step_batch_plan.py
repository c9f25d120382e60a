"""Host planning of the one-launch batch step (no device): the time-step
chain planned for a batch, its workspace and plan record, and what it
refuses."""
import pytest

from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs


@pytest.mark.parametrize("dtype,es", [(H.F64, 8), (H.F32, 4)])
def test_step_chain_plans_one_launch_for_a_batch(dtype, es):
    sizes = [(64, 64), (1, 1), (300, 5), (191, 4)]
    c = H.Chain(H.euler_step_spec(dtype=dtype, with_smax=True))
    info = c.plan_batch(sizes, precision=H.PREC_F32_F64ACC if dtype == H.F32 else H.PREC_NATIVE)
    assert H.FAMILY[info.family] == "euler_xy" and info.fused
    total = sum(nx * ny for nx, ny in sizes)
    plane = (total * es + 255) // 256 * 256
    assert info.workspace_bytes == 4096 + 4 * plane
    b = c.plan_json()["batch"]
    assert b["one_launch_step"] == 1 and b["workspace_bytes"] == info.workspace_bytes
    assert b["grids"] == len(sizes) and b["y_seg"] == [15] * len(sizes)
    assert [c.batch_offset(g) for g in range(len(sizes))] == [0, 4096, 4097, 5597]


def test_step_batch_segments_from_a_forced_configuration():
    c = H.Chain(H.euler_step_spec(with_smax=True))
    c.plan_batch(inputs.batch_sizes(5, seed=1, lo=8, hi=64), config_source=H.CONFIG_FORCED,
                 forced=(256, 1, 7, 3, 0))
    assert c.plan_json()["batch"]["y_seg"] == [7] * 5


def test_step_batch_refusals():
    c = H.Chain(H.euler_step_spec(with_smax=True))
    for g, a in zip(H.EULER_GOALS, H.EULER_AXIOMS):
        c.alias(g, a)
    with pytest.raises(H.HfavError) as e:
        c.plan_batch([(64, 64)])
    assert e.value.code == H.EUNSUP
    d = H.Chain(H.euler_step_spec(with_smax=True))
    with pytest.raises(H.HfavError) as e:
        d.plan_batch([(64, 64)] * 641)
    assert e.value.code == H.EINVAL
    d.plan_batch([(64, 64)])
    # the workspace is required
    assert d.execute_status([1, 2, 3, 4, 5], [6, 7, 8, 9, 10]) == H.ENOPLAN
