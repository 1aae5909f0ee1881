"""The kernel_timing option brackets every k-th span-step launch with HIP events.

The timed launches are counted in the result, the designs are unchanged, and a negative period
is rejected when the context is created."""
import pytest

import sdinputs as S

pytestmark = pytest.mark.gpu


def test_sampled_kernel_timing(params_path, weights):
    import paper_2609_32308_amd as sd
    gp, gt = sd.Params(params_path), sd.CodonTable(weights)
    p = S.protein(40, 3)
    base = sd.Context(0)
    r0 = base.design(p, gt, gp, 4.0)
    base.close()
    assert r0.n_timed_launches == 0 and r0.t_span_kernels_s == 0.0
    for k in (1, 7, 16):
        print("kernel_timing", k, flush=True)
        c = sd.Context(0, kernel_timing=k)
        r = c.design(p, gt, gp, 4.0)
        c.close()
        n = r.n_span_launches
        assert n == r0.n_span_launches > 0
        assert r.n_timed_launches == (n + k - 1) // k
        assert r.t_span_kernels_s > 0.0
        assert (r.energy, r.objective_fixed, r.mrna, r.structure) == (r0.energy, r0.objective_fixed, r0.mrna, r0.structure)
    with pytest.raises(sd.SDError) as e:
        sd.Context(0, kernel_timing=-1)
    assert e.value.code == -1
