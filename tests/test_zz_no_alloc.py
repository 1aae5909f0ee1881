"""sd_design_noalloc (the design entry point that allocates nothing: its device state lives in the
library's static scratch array) against sd_design through the C ABI: identical results on two
calls in a row, the second with a smaller input, at both lambdas and after a switch of the
parameter set; a design too large for the array is rejected with SD_E_NOMEM."""
import pytest

import sdinputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def sd():
    import paper_2609_32308_amd as m
    return m


def full(r):
    return (r.energy, r.objective_fixed, r.fixed_shift, r.mrna, r.structure, r.codon_cost, r.objective_kcal,
            r.cai, r.n_states, r.n_cells, r.n_candidates, r.n_visits, r.n_feasible, r.cand_slots, r.path)


def test_noalloc_equals_design_on_consecutive_calls(sd, params_path, weights, tmp_path):
    ctx = sd.Context(0)
    gt = sd.CodonTable(weights)
    gp = sd.Params(params_path)
    other = str(tmp_path / "other.par")
    S.write_params(other, S.synthetic_params(seed=2005))
    gp2 = sd.Params(other)
    # larger then smaller input, both lambdas, then the other parameter set and back
    calls = [(S.protein(160, 3), 4.0, gp), (S.protein(45, 4), 0.0, gp), (S.protein(90, 5), 4.0, gp2),
             (S.protein(30, 6), 0.0, gp2), (S.protein(120, 7), 0.0, gp)]
    for p, lam, P in calls:
        say("noalloc", len(p), lam)
        a = ctx.design_noalloc(p, gt, P, lam)
        b = ctx.design(p, gt, P, lam)
        assert full(a) == full(b)
        assert a.path == sd.PATH_PLAIN and a.n_span_launches == 3 * len(p)
    ctx.close()


def test_noalloc_rejects_a_design_beyond_the_array(sd, params_path, weights):
    ctx = sd.Context(0)
    gt, gp = sd.CodonTable(weights), sd.Params(params_path)
    with pytest.raises(sd.SDError) as e:
        ctx.design_noalloc(S.protein(1976, 1), gt, gp, 0.0)
    assert e.value.code == -7 and "static" in str(e.value)
    # the array still serves the next call
    p = S.protein(50, 2)
    assert full(ctx.design_noalloc(p, gt, gp, 4.0)) == full(ctx.design(p, gt, gp, 4.0))
    ctx.close()
