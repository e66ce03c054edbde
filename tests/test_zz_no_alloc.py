"""The product that allocates nothing (pbt_matvec_dev_static) against the
product of pbt_matvec_dev, through the C ABI.

Both run the same kernels in the same order on the same system; only the
addresses of the work vectors and partial sums differ (the library's static
scratch array instead of the context's buffers), so the results must be
bitwise equal, in FP64 and with FP32 interactions.  Two systems in a row,
the second smaller, share the scratch array: the second call must not see
anything of the first.
"""
import numpy as np
import pytest
import torch

from paper_1506_03745_amd import FP64, MIXED, PbtError, from_problem
from tests.gpu_cases import case
from workloads.problems import config_problem

pytestmark = pytest.mark.gpu


def _both(s, x, prec):
    xd = torch.tensor(x, device="cuda:0")
    y_ref = torch.empty_like(xd)
    y_static = torch.full_like(xd, float("nan"))
    s.matvec_dev(xd, y_ref, prec=prec)
    s.matvec_dev_static(xd, y_static, prec=prec)
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y_static.cpu().numpy()


def test_static_product_equals_matvec_dev_on_two_systems():
    big, _ = from_problem(case("stern_plate"), treecode=1, ncrit=40, theta=0.5, taylor_p=6)
    small, _ = from_problem(config_problem("kirkwood", level=1), treecode=1, ncrit=20, theta=0.5, taylor_p=4)
    big.prepare()
    small.prepare()
    assert small.num_unknowns() < big.num_unknowns()
    for s, seed in ((big, 1), (small, 2), (big, 3)):
        x = np.random.default_rng(seed).standard_normal(s.num_unknowns())
        for prec in (FP64, MIXED):
            y_ref, y_static = _both(s, x, prec)
            assert np.all(np.isfinite(y_static))
            assert np.array_equal(y_ref, y_static), (seed, prec)
    big.close()
    small.close()


def test_static_product_of_the_large_twin_and_an_unprepared_system():
    """A system of 13312 unknowns (the large workload's twin, autotuned
    launch shape) fits the scratch array; an unprepared system is refused."""
    s, _ = from_problem(config_problem("star_plate_twin"), prec=MIXED, theta=0.5, taylor_p=6, ncrit=300)
    s.prepare()
    s.autotune()
    x = np.random.default_rng(5).standard_normal(s.num_unknowns())
    for prec in (MIXED, FP64):
        y_ref, y_static = _both(s, x, prec)
        assert np.array_equal(y_ref, y_static)
    s.close()
    u, _ = from_problem(case("kirkwood_l1"), treecode=0)
    xd = torch.zeros(u.num_unknowns(), dtype=torch.float64, device="cuda:0")
    with pytest.raises(PbtError, match="STATE"):
        u.matvec_dev_static(xd, torch.empty_like(xd))
    u.prepare()
    u.matvec_dev_static(xd, torch.empty_like(xd))
    u.close()
