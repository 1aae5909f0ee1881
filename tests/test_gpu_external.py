"""Contexts on caller-owned device memory and streams (sd_context_create_external).

A PyTorch uint8 tensor serves as the device pool and a PyTorch stream as the stream, the
plumbing the library is meant to share with a framework.  Plain, batched (graph-captured on the
caller's stream) and forbidden-motif designs must be identical to those of a library-owned
context; the library must write into the caller's pool, report SD_E_NOMEM when a design does not
fit, reject pools that are not aligned device memory, and leave pool and stream alive when the
context is destroyed.

PyTorch and the library each ship a HIP runtime with the same soname, and a process loads only
the first: torch works when it is imported before the library (the library then runs on torch's
runtime), not after.  Earlier tests of this session have loaded the library already, so the
checks run in a fresh child process that imports torch first.
"""
import os
import subprocess
import sys

import pytest

import sdinputs as S

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def say(*a):
    print(*a, flush=True)


def key(r):
    return (r.energy, r.objective_fixed, r.mrna, r.structure, r.n_candidates, r.n_visits)


def test_external_pool_and_stream():
    code = ("import torch, sys; sys.path[:0] = [%r, %r]; import test_gpu_external as t; t.interop()"
            % (ROOT, HERE))
    say("external: child process (torch first)")
    r = subprocess.run([sys.executable, "-u", "-c", code], capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr[-3000:], flush=True)
    assert r.returncode == 0
    assert "interop ok" in r.stdout


def interop():
    import torch  # before the library: one HIP runtime for both
    import paper_2609_32308_amd as sd
    gp = sd.Params(S.default_params_path())
    gt = sd.CodonTable(S.codon_weights(2026))
    p = S.protein(120, 4)
    batch = [S.protein(A, 500 + i) for i, A in enumerate((40, 75, 130, 60))]
    lams = [0.0, 4.0, 0.0, 4.0]
    motifs = S.motifs(8, 41)
    say("external: reference designs")
    own = sd.Context(0)
    ref = [own.design(p, gt, gp, lam) for lam in (0.0, 4.0)]
    refb = own.design_batch(batch, lams, gt, gp)
    refm = own.design_motifs(p, motifs, gt, gp, 4.0)
    own.close()

    pool = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.Stream(device=0)
    torch.cuda.synchronize()
    say("external: designs in a torch pool on a torch stream")
    ctx = sd.Context.external(stream.cuda_stream, pool.data_ptr(), pool.numel())
    for lam, r0 in zip((0.0, 4.0), ref):
        assert key(ctx.design(p, gt, gp, lam)) == key(r0)
    assert [key(r) for r in ctx.design_batch(batch, lams, gt, gp)] == [key(r) for r in refb]
    assert key(ctx.design_motifs(p, motifs, gt, gp, 4.0)) == key(refm)
    torch.cuda.synchronize()
    assert int(pool[: 1 << 20].count_nonzero()) > 0  # the tables live in the caller's pool

    say("external: a pool too small for the design")
    small = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    c2 = sd.Context.external(stream.cuda_stream, small.data_ptr(), small.numel())
    with pytest.raises(sd.SDError) as e:
        c2.design(S.protein(300, 1), gt, gp, 0.0)
    assert e.value.code == -7
    c2.close()
    ctx.close()
    # pool and stream still belong to the caller and stay usable
    with torch.cuda.stream(stream):
        pool[:16].fill_(7)
    torch.cuda.synchronize()
    assert int(pool[:16].sum()) == 7 * 16

    say("external: invalid pools")
    for ptr, nbytes in ((0, 1 << 20), (pool.data_ptr() + 8, 1 << 20), (pool.data_ptr(), 1024)):
        with pytest.raises(sd.SDError) as e:
            sd.Context.external(stream.cuda_stream, ptr, nbytes)
        assert e.value.code == -1
    host = torch.zeros(1 << 20, dtype=torch.uint8)
    with pytest.raises(sd.SDError) as e:
        sd.Context.external(stream.cuda_stream, host.data_ptr(), host.numel())
    assert e.value.code == -1
    say("interop ok")
