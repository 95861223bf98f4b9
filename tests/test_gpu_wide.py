"""GPU parity for wide leading subspaces, d_r > 128 (needs an MI355X).

These are the shapes of the paper's IVF-RaBitQ comparison (d_r = D: no residual terms, Section 6 Exp-1)
and of its choice-of-d study (Section 5.3 Eq 8, Exp-4: d up to 512).  Each takes code paths that the
d_r <= 128 tests never reach:
  * d_r in (128, 192]: the 4-slice scan with query levels padded to 256 bytes;
  * d_r > 256: the scan with any number of K slices (its operands loaded from global memory), seed passes
    of 16, 32 and 48 code words per row, and the pair code with 8, 16 and 24 dimensions per lane;
  * B = 4 extended codes at those widths.
Small synthetic data sets (a Gaussian mixture with a power-law spectrum) keep the oracle's FP64 import
and row checks fast; every result row is checked against the oracle (tests/parity.py).
"""
import os
import tempfile

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("no GPU", allow_module_level=True)

import torch  # noqa: E402

import oracle  # noqa: E402
import paper_2411_06158_amd as mrq  # noqa: E402
from paper_2411_06158_amd import synth  # noqa: E402
from parity import assert_rows, check_rows  # noqa: E402


def _env(D, d, B, N, nq=40, nlist=32, seed=11):
    print(f"\n[gpu] wide: build N={N} D={D} d={d} B={B} nlist={nlist}", flush=True)
    m = synth.build_model(synth.MixtureSpec(D=D, n_comp=32, decay=1.0, cluster_dims=8, model_seed=seed))
    X, Q = synth.sample(m, N, 1), synth.sample(m, nq, 2)
    ix = mrq.Index.build(torch.from_numpy(X).cuda(), d_r=d, bits=B, nlist=nlist)
    path = os.path.join(tempfile.mkdtemp(), "ix.mrqx")
    ix.export(path)
    orc = oracle.Index.load_export(path, X)
    return dict(X=X, Q=Q, Qd=torch.from_numpy(Q).cuda(), ix=ix, orc=orc, path=path)


def _check(env, k, nprobe, **kw):
    ids, dists = env["ix"].search(env["Qd"], k, nprobe, **kw)
    torch.cuda.synchronize()
    prm = oracle.params(**{a: b for a, b in kw.items() if a in ("bq", "stage2", "use_ext")})
    st = check_rows(env["orc"], env["X"], env["Q"], ids.cpu().numpy(), dists.cpu().numpy(), k, nprobe, prm)
    assert_rows(st, f"D={env['X'].shape[1]} d={env['orc'].d} k={k} nprobe={nprobe} {kw}")
    return ids


# (D, d, B, N): the code widths these reach are noted per case
WIDE = [
    (256, 192, 1, 8000),    # KI = 3 (4-slice scan, padded levels), WP = 8
    (256, 192, 4, 8000),
    (512, 320, 1, 6000),    # any-K scan (5 slices), WP = 16, pair code 8 dims per lane
    (512, 320, 4, 6000),
    (512, 384, 1, 6000),    # 6 slices, WP = 16
    (512, 512, 1, 6000),    # d = D: no tail (IVF-RaBitQ shape), 8 slices
    (512, 512, 4, 6000),
    (960, 960, 1, 5000),    # the GIST shape of the IVF-RaBitQ comparison: WP = 32, 15 slices, 16 dims per lane
    (1536, 1536, 1, 3000),  # the largest d_r: WP = 48, 24 slices, 24 dims per lane
]


@pytest.mark.parametrize("D,d,B,N", WIDE)
def test_wide_leading_dims_match_oracle(D, d, B, N):
    env = _env(D, d, B, N)
    try:
        assert env["ix"].d == d
        if d == D:  # no residual subspace: the tail norms and eps_r vanish (the d = D special case)
            assert np.abs(oracle.Index.load_export(env["path"]).get("tx")).max() == 0
        ids = _check(env, 10, 8)
        assert (ids[:, 0] >= 0).all()
        _check(env, 50, 16)
        _check(env, 10, 8, stage2=False)
        if B > 1:
            _check(env, 10, 8, use_ext=False)
    finally:
        env["ix"].close()


def test_wide_per_query_path_and_groups_bit_identical():
    """At d = 320 (any-K scan) the per-query path and every query-group size give bit-identical rows."""
    env = _env(512, 320, 4, 6000, nq=30)
    try:
        ix, Qd = env["ix"], env["Qd"]
        a_i, a_d = ix.search(Qd, 10, 12)
        for kw in (dict(mode=mrq.MRQ_PER_QUERY), dict(group=32), dict(group=64), dict(exact_cap=1)):
            b_i, b_d = ix.search(Qd, 10, 12, **kw)
            torch.cuda.synchronize()
            assert torch.equal(a_i, b_i), kw
            assert torch.equal(a_d.view(torch.int32), b_d.view(torch.int32)), kw
    finally:
        env["ix"].close()
