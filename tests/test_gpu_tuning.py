"""Tuning cache file: the settled batch schedules and span tiles of one context, saved to a text
file and loaded into a new context, make that context's first designs run the saved choices
without exploring, with the same designs; a file that is malformed, written for another device
or names a schedule the library cannot run is refused whole."""
import pytest

import sdinputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def sd():
    import paper_2609_32308_amd as m
    return m


@pytest.fixture(scope="module")
def env(sd, params_path, weights):
    return sd.Params(params_path), sd.CodonTable(weights)


def key(r):
    return (r.energy, r.objective_fixed, r.mrna, r.structure, r.n_candidates, r.n_visits)


def sched(rb):
    s = {(r.sched_threads, r.sched_grid, r.sched_item_waves, r.sched_tuned) for r in rb}
    assert len(s) == 1
    return s.pop()


@pytest.fixture(scope="module")
def batch():
    prots = [S.protein(30 + 7 * i, 700 + i) for i in range(16)]
    lams = [0.0 if i % 2 == 0 else 4.0 for i in range(len(prots))]
    return prots, lams


@pytest.fixture(scope="module")
def saved(sd, env, batch, tmp_path_factory):
    # a context that has settled one batch class and one plain length class, and its file
    gp, gt = env
    prots, lams = batch
    c = sd.Context(0)
    for k in range(10):
        say("tuning batch call", k)
        rb = c.design_batch(prots, lams, gt, gp)
        if sched(rb)[3] == 1:
            break
    assert sched(rb)[3] == 1
    p = S.protein(90, 5)
    for k in range(5):
        say("tuning plain design", k)
        r = c.design(p, gt, gp, 0.0)
    assert r.sched_tuned == 1
    path = tmp_path_factory.mktemp("tuning") / "sd.tuning"
    c.tuning_save(path)
    out = dict(file=path, text=path.read_text(), batch_keys=[key(x) for x in rb], batch_sched=sched(rb),
               plain=(p, key(r)))
    c.close()
    say(out["text"])
    return out


def test_saved_file_layout(saved):
    lines = saved["text"].splitlines()
    assert lines[0] == "sparsedesign-tuning 1"
    dev = lines[1].split()
    assert dev[:2] == ["device", "gfx950"] and int(dev[2]) > 0
    batch = [x.split() for x in lines[2:] if x.startswith("batch ")]
    span = [x.split() for x in lines[2:] if x.startswith("span ")]
    assert len(batch) == 1 and len(span) >= 3 and len(batch) + len(span) == len(lines) - 2
    threads, grid, iw = saved["batch_sched"][:3]
    assert [int(v) for v in batch[0][2:]] == [grid, threads, iw]
    for s in span:
        assert (int(s[3]), int(s[4])) in ((1024, 16), (512, 8), (256, 4), (256, 1))
        assert 0 <= int(s[2]) < 16 and int(s[1]) == 8  # floor log2 of 270 nucleotides


def test_loaded_context_runs_saved_choices_at_once(sd, env, batch, saved):
    gp, gt = env
    prots, lams = batch
    c = sd.Context(0)
    c.tuning_load(saved["file"])
    rb = c.design_batch(prots, lams, gt, gp)
    assert sched(rb) == saved["batch_sched"]
    assert [key(r) for r in rb] == saved["batch_keys"]
    p, k = saved["plain"]
    r = c.design(p, gt, gp, 0.0)
    assert r.sched_tuned == 1 and key(r) == k
    # saving the loaded context writes the same choices
    again = saved["file"].parent / "again.tuning"
    c.tuning_save(again)
    assert again.read_text() == saved["text"]
    c.close()


def _bad_files(text):
    lines = text.splitlines()
    head, dev, body = lines[0], lines[1].split(), lines[2:]
    cus = int(dev[2])
    b = next(x for x in body if x.startswith("batch ")).split()
    return {
        "header": "\n".join(["sparsedesign-tuning 2", lines[1]] + body),
        "device_cus": "\n".join([head, f"device gfx950 {cus + 8}"] + body),
        "device_arch": "\n".join([head, f"device gfx942 {cus}"] + body),
        "threads": "\n".join(lines + [f"batch 99 {cus} 128 2"]),
        "grid": "\n".join(lines + [f"batch 99 {cus * 1000} 256 1"]),
        "grid_not_per_cu": "\n".join(lines + [f"batch 99 {cus + 1} 256 1"]),
        "span_tile": "\n".join(lines + ["span 6 3 768 12"]),
        "span_band": "\n".join(lines + ["span 6 16 256 4"]),
        "kind": "\n".join(lines + ["tile 6 3 256 4"]),
        "short": "\n".join(lines + [" ".join(b[:4])]),
        "empty": "",
    }


def test_bad_files_are_refused_whole(sd, env, batch, saved):
    gp, gt = env
    prots, lams = batch
    c = sd.Context(0)
    for name, text in _bad_files(saved["text"]).items():
        f = saved["file"].parent / f"bad_{name}.tuning"
        f.write_text(text + "\n")
        say("bad file", name)
        with pytest.raises(sd.SDError) as e:
            c.tuning_load(f)
        assert e.value.code == -1, name  # SD_E_ARG
    with pytest.raises(sd.SDError) as e:
        c.tuning_load(saved["file"].parent / "missing.tuning")
    assert e.value.code == -1
    # nothing was installed: the batch class and the plain class still explore
    assert sched(c.design_batch(prots, lams, gt, gp))[3] == 0
    assert c.design(saved["plain"][0], gt, gp, 0.0).sched_tuned == 0
    c.close()


def test_fresh_context_saves_an_empty_tuning_file(sd, env, batch, tmp_path):
    # nothing settled: the file holds only the header and the device line, and loading it leaves
    # every class exploring
    gp, gt = env
    prots, lams = batch
    c = sd.Context(0)
    f = tmp_path / "empty.tuning"
    c.tuning_save(f)
    lines = f.read_text().splitlines()
    assert len(lines) == 2 and lines[0] == "sparsedesign-tuning 1" and lines[1].startswith("device gfx950 ")
    c2 = sd.Context(0)
    c2.tuning_load(f)
    assert sched(c2.design_batch(prots, lams, gt, gp))[3] == 0
    c2.close()
    c.close()
