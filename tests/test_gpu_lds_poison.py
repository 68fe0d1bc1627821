"""The LDS-poisoned debug build (every kernel fills its LDS with NaN before first use) gives the
same outputs as the release build on every kernel family that holds LDS, so no kernel reads an
LDS word that was not written in the same launch (padding words, a wrong stride, a tail tile)."""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_poisoned_build_matches_release():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_07042_amd as ax
    from paper_2504_07042_amd import build as hipbuild
    assert os.path.exists(hipbuild.LIB_POISON), "the LDS-poisoned twin is built by __graft_entry__.build()"
    assert os.path.realpath(ax.LIBPATH) != os.path.realpath(hipbuild.LIB_POISON)
    sys.path.insert(0, HERE)
    import lds_poison_cases
    ref = lds_poison_cases.run_all()
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "poison.npz")
        env = dict(os.environ, AXHOSFEM_LIB=hipbuild.LIB_POISON)
        print(f"[lds-poison] child on {hipbuild.LIB_POISON}", flush=True)
        r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "lds_poison_cases.py"), out], env=env,
                           timeout=300, capture_output=True, text=True)
        print(r.stdout[-3000:], r.stderr[-3000:], flush=True)
        assert r.returncode == 0, r.stderr[-2000:]
        got = dict(np.load(out))
    assert sorted(got) == sorted(ref)
    bad, inexact = [], []
    for name, Yr in ref.items():
        Yp = got[name]
        if not np.isfinite(Yp).all():
            bad.append(f"{name}: {np.count_nonzero(~np.isfinite(Yp))} non-finite")
        elif not np.array_equal(Yp, Yr):
            scale = np.abs(Yr).max()
            d = np.abs(Yp.astype(np.float64) - Yr).max() / scale
            (bad if d > 1e-5 else inexact).append(f"{name}: max rel diff {d:.2e}")
    print(f"[lds-poison] {len(ref)} cases, {len(inexact)} not bit-identical: {inexact[:8]}", flush=True)
    assert np.isfinite(np.concatenate([v.ravel() for v in ref.values()])).all()
    assert not bad, bad
