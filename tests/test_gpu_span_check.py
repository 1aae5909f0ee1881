"""Span-check debug mode (race detection): every plain span step is run a second time, with
another workgroup size, from restored committed counts, and digests of what the two runs wrote
must agree; a batch is re-run under another persistent schedule and each member's table digest
must agree.  Designs are unchanged by the mode.  Mode 2 deliberately skips restoring the visit
counters before the re-run, so the comparison must report the first span."""
import pytest

import oracle as O
import sdinputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def sd():
    import paper_2609_32308_amd as m
    return m


def key(r):
    return (r.energy, r.objective_fixed, r.mrna, r.structure, r.n_candidates, r.n_visits, r.n_feasible)


def test_plain_span_check_is_clean_and_leaves_designs(sd, params_path, weights, oparams):
    gt, gp = sd.CodonTable(weights), sd.Params(params_path)
    chk, ref = sd.Context(0, span_check=1), sd.Context(0)
    for A, seed, lam in ((20, 1, 0.0), (41, 3, 4.0), (90, 5, 4.0)):
        p = S.protein(A, seed)
        say("span check", A, lam)
        r = chk.design(p, gt, gp, lam)
        assert key(r) == key(ref.design(p, gt, gp, lam))
        d = O.design(p, weights, oparams, lam)
        assert (r.energy, r.objective_fixed, r.mrna, r.structure) == (d.energy, d.objective_fixed, d.mrna, d.structure)
    chk.close()
    ref.close()


def test_span_check_reports_a_difference(sd, params_path, weights):
    gt, gp = sd.CodonTable(weights), sd.Params(params_path)
    c = sd.Context(0, span_check=2)
    with pytest.raises(sd.SDError) as e:
        c.design(S.protein(20, 1), gt, gp, 0.0)
    assert e.value.code == -11 and "span check: span" in str(e.value)
    c.close()


def test_batch_span_check_is_clean(sd, params_path, weights):
    gt, gp = sd.CodonTable(weights), sd.Params(params_path)
    prots = [S.protein(A, 900 + i) for i, A in enumerate((12, 33, 57, 21, 70, 44))]
    lams = [0.0, 4.0, 0.0, 4.0, 4.0, 0.0]
    chk, ref = sd.Context(0, span_check=1), sd.Context(0)
    rb = chk.design_batch(prots, lams, gt, gp)
    rr = ref.design_batch(prots, lams, gt, gp)
    for a, b in zip(rb, rr):
        assert key(a) == key(b) and a.path == sd.PATH_PERSISTENT
    chk.close()
    ref.close()


def test_span_check_option_validated(sd):
    with pytest.raises(sd.SDError) as e:
        sd.Context(0, span_check=3)
    assert e.value.code == -1
