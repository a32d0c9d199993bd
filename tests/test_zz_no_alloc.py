"""asm_plan_vjp_noalloc, the VJP entry point that allocates nothing, against asm_plan_vjp:
the same kernels on the same moments, so the results agree bit for bit; two plans in a row,
the second smaller, share the library's per-device scratch array."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_01379_amd as pk
    return pk


def _compare(pk, plan, v):
    import torch
    g_ref, se_ref = plan.vjp(v, stderr=True)
    out = torch.full_like(g_ref, float("nan"))
    se = torch.full_like(se_ref, float("nan"))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan.vjp_noalloc(v, out, se)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert torch.equal(out, g_ref)
    assert torch.equal(se, se_ref)
    # without the error bar
    out2 = torch.full_like(g_ref, float("nan"))
    plan.vjp_noalloc(v, out2)
    torch.cuda.synchronize()
    assert torch.equal(out2, g_ref)
    return free0, free1


def test_noalloc_vjp_equals_vjp_on_two_plans_in_a_row(pk):
    import torch
    dev = torch.device("cuda:0")
    # first call: the single-continuation problem (201 data points, 800 grid points), float32 two-role plan
    big = workloads.single_continuation()
    plan = pk.Plan([big], chains=1024, burnin=50, sweeps=200, seed=3, precision="fp32", groups=32,
                   want_vjp=True, start="nnls")
    plan.run()
    v = torch.as_tensor(workloads.differentiation_cotangent(big.N), dtype=torch.float64, device=dev)
    _compare(pk, plan, v)
    plan.close()
    # second call, smaller: 41 data points, 48 grid points, float64, 8 groups
    small = workloads.small_problem(M=41, N=48, nblocks=3, sigma=2e-3)
    plan = pk.Plan([small], chains=64, burnin=20, sweeps=300, seed=4, precision="fp64", groups=8,
                   want_vjp=True)
    plan.run()
    v = torch.linspace(-1.0, 1.0, small.N, dtype=torch.float64, device=dev)
    free0, free1 = _compare(pk, plan, v)
    assert free1 == free0, (free0, free1)   # no device memory taken by the call
    plan.close()


def test_noalloc_vjp_refuses_what_it_cannot_hold(pk):
    """(4 groups + 2) x sum M + 2 x problems x groups doubles above 2^23: a clear error, and
    the allocating entry point still serves the plan."""
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    probs = []
    for j in range(300):   # 300 problems of 120 data points: 258 x 36000 > 2^23 with 64 groups
        M, N = 120, 8
        K = np.exp(-np.outer(np.linspace(0, 4, M), np.linspace(0.1, 3, N)))
        probs.append(workloads.Problem(K=K, G=K @ rng.uniform(0.5, 1.5, N), sigma=np.full(M, 1e-2),
                                       block_start=np.array([0, N], np.int64)))
    plan = pk.Plan(probs, chains=64, burnin=0, sweeps=10, seed=6, precision="fp64", groups=64, want_vjp=True)
    plan.run()
    v = torch.ones(8 * 300, dtype=torch.float64, device=dev)
    out = torch.empty(120 * 300, dtype=torch.float64, device=dev)
    with pytest.raises(pk.AsmError) as e:
        plan.vjp_noalloc(v, out)
    assert "scratch" in str(e.value)
    g = plan.vjp(v)
    assert torch.isfinite(g).all()
    plan.close()


def test_noalloc_vjp_needs_a_run(pk):
    import torch
    p = workloads.small_problem(M=41, N=48, nblocks=3, sigma=2e-3)
    plan = pk.Plan([p], chains=64, burnin=0, sweeps=10, precision="fp64", groups=8, want_vjp=True)
    v = torch.ones(p.N, dtype=torch.float64, device="cuda:0")
    out = torch.empty(p.K.shape[0], dtype=torch.float64, device="cuda:0")
    with pytest.raises(pk.AsmError):
        plan.vjp_noalloc(v, out)
    plan.close()
