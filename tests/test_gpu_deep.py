"""Single-trial parity at depth: T = 520 queries at n = 40037 (FP32),
beyond the 512 reflectors up to which the data pass forms z = T'w in its
prologue and the Gaussian random pass takes the reflector step in its
prologue, so both the fused prologues (k <= 512) and their separate-kernel
fallbacks (k > 512) answer queries.

One fixed sequence of query vectors with unit-scale entries, mixing Q and Q',
goes to three handles with the same key, one per launch shape (workgroups of
1, 2 and 4 chunks of 256 rows, forced through HD_CPT); the FP64 oracle
answers the same sequence once and every answer of every handle is compared
with it (mode B, 1e-4).

Where a data-side pivot of some handle is a near tie (|p_k| / ||p[k:]|| below
KAPPA), FP32 rounding may legitimately pick the other sign (a different but
equally valid orthogonal completion); the oracle then follows the handles'
sign, which must agree among them.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2101_07464_amd as hd  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
KAPPA = 1e-5
T = 520


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _pattern(ens):
    if ens == "haar":
        return [t % 3 == 1 for t in range(T)]
    # Gaussian: mostly Q' queries, so the L side passes 512 reflectors as
    # the data side (queries up to 517) and as the random side of the last
    # three Q-queries
    return [not (q in (1, 2, 200) or q >= 518) for q in range(1, T + 1)]


def _data_index(ens, flags):
    """(side, reflector index) of the data-side reflector of each query."""
    out, r, l = [], 0, 0
    for q, tr in enumerate(flags):
        side = 1 if tr else 0
        if ens == "haar":
            out.append((side, q))
        else:
            out.append((side, l if tr else r))
            if tr:
                l += 1
            else:
                r += 1
    return out


@pytest.fixture
def restore_env():
    old = os.environ.get("HD_CPT")
    hd.autotune_clear()
    yield
    if old is None:
        os.environ.pop("HD_CPT", None)
    else:
        os.environ["HD_CPT"] = old


@pytest.mark.parametrize("ens", ["haar", "gaussian"])
def test_deep_trajectory_all_shapes_against_oracle(restore_env, ens):
    n = 40037
    m = n if ens == "haar" else 36011
    E = hd.HAAR if ens == "haar" else hd.GINIBRE
    EO = oracle.HAAR if ens == "haar" else oracle.GINIBRE
    sig = 1.0 if ens == "haar" else 1.0 / np.sqrt(m)
    flags = _pattern(ens)
    rng = np.random.default_rng(520)
    xs = [rng.standard_normal(m if tr else n).astype(np.float32)
          for tr in flags]
    answers, piv = {}, {}
    for cpt in (1, 2, 4):
        os.environ["HD_CPT"] = str(cpt)
        assert hd.shape_rule(E, n) == cpt
        A = hd.LazyMatrix(E, n, m=m, t_max=T, seed=11, trial=3, sigma=sig,
                          device=DEV)
        ys = []
        for x, tr in zip(xs, flags):
            xt = torch.from_numpy(x).to(DEV)
            ys.append(A.rmv(xt) if tr else A.mv(xt))
        torch.cuda.synchronize()
        assert A.status() == 0
        answers[cpt] = [y.double().cpu().numpy() for y in ys]
        piv[cpt] = (A.pivots(0), A.pivots(1))
        print("deep %s: cpt %d done" % (ens, cpt), flush=True)
        A.close()
    orc = oracle.HDOracle(EO, n, m=m, tmax=T, seed=11, trial=3, sigma=sig)
    forced = 0
    for side, idx in _data_index(ens, flags):
        signs = set()
        near = False
        for cpt in (1, 2, 4):
            nu, pv, sg = piv[cpt][side]
            if nu[idx] > 0 and abs(pv[idx]) / nu[idx] < KAPPA:
                near = True
            signs.add(int(sg[idx]))
        if near:
            assert len(signs) == 1, (side, idx, signs)
            orc.force_sign(side, idx + 1, signs.pop())
            forced += 1
    ref = oracle.replay(orc, [x.astype(np.float64) for x in xs], flags)
    worst = {}
    for cpt in (1, 2, 4):
        errs = [relerr(y, r) for y, r in zip(answers[cpt], ref)]
        worst[cpt] = (max(errs), int(np.argmax(errs)) + 1)
        assert max(errs) < 1e-4, (cpt, worst[cpt])
    print("deep %s: worst per shape %s, forced signs %d" %
          (ens, worst, forced))
