"""Where IBIP and the opening disagree at equal saturation (Section 3.1.1,
Figures 6 and 8), pinned on the oracle.

Let T be an opening level, MIO_T = {mio_r2 >= T} (every opening at a level
>= T), m = |MIO_T|, k_eq the last IBIP step whose cumulative count is <= m,
IBIP_eq = {0 < seq <= k_eq}, and k*(T) the first step with M_k < T. Then:

* IBIP's configuration before k*(T), C_T = {0 < seq < k*(T)}, contains MIO_T:
  its centres are exactly the opening's kept centres (the seed-set invariant)
  and each paints its own ball, whose squared radius is at least T. This is
  the peak-pressure envelope of Section 2.2.2: at the pressure of T, IBIP
  holds at least the opening's voxels.
* a = |IBIP_eq \\ MIO_T| are voxels IBIP holds through balls larger than the
  opening's (every centre of a step <= k_eq is a kept centre); b = |MIO_T \\
  IBIP_eq| are opening voxels whose kept centres IBIP has not reached at
  equal count (a reached centre would have painted them). Since |IBIP_eq| <=
  m, b = a + gap with gap = m - |IBIP_eq| < (size of step k_eq + 1), and the
  symmetric difference is 2a + gap.
* In the continuum a maximal ball B(c, dt(c)) is the union of balls of radius
  sqrt(T) whose centres lie in the same component of {dt >= sqrt(T)}, so a = 0;
  on the lattice that union misses voxels near the ball's edge. The measured
  a therefore falls with the resolution of one geometry (disks rendered at 1
  and 2 pixels per unit: max a from 0.38 % to 0.16 % of the pore pixels; at
  1, 2 and 4 pixels per unit on a 500-unit box 0.23 %, 0.13 %, 0.08 %).

The soft bound of 0.5 % of the pore space applies to a, the part
that depends on the method: both 500 x 500 images stay below it (0.37 % and
0.27 %); the symmetric difference counts each such voxel twice and adds the
step granularity gap.
"""
import numpy as np
import pytest

import oracle
from paper_2101_03240_amd import synth


def _levels(img, inl, T=None):
    r = oracle.invade(img, inl)
    seq, M, K = r["seq"], r["M"], r["K"]
    if T is None:
        T = np.unique(M)[::-1].astype(np.uint32)
        T = T[T >= 1]
    T = np.asarray(T, dtype=np.uint32)
    po = oracle.mio(img, inl, T)
    mio = po["mio_r2"]
    cnt = np.bincount(seq[seq > 0], minlength=K + 1)[1:].astype(np.int64)
    cum = np.cumsum(cnt)
    s = oracle.steps(seq, M)
    sm = oracle.satmap(seq, s["sat"])
    dis = oracle.compare_opening(sm, mio, T, po["mio_sat"])["disagree"]
    rows = []
    for i, t in enumerate(T):
        mio_t = mio >= t
        m = int(mio_t.sum())
        keq = int(np.searchsorted(cum, m, side="right"))
        ibip_eq = (seq > 0) & (seq <= keq)
        below = np.nonzero(M < t)[0]
        kstar = int(below[0]) + 1 if below.size else K + 1
        conf = (seq > 0) & (seq < kstar)
        rows.append(dict(T=int(t), m=m, keq=keq, kstar=kstar, a=int((ibip_eq & ~mio_t).sum()),
                         b=int((mio_t & ~ibip_eq).sum()), gap=m - (int(cum[keq - 1]) if keq else 0),
                         next_step=int(cnt[keq]) if keq < K else 0, dis=int(dis[i]),
                         mio_in_conf=bool((conf | ~mio_t).all()), eq_in_conf=bool((conf | ~ibip_eq).all()),
                         excess=int(conf.sum()) - m))
    return rows, int((img > 0).sum())


def _image(kind):
    if kind == "noise":
        return synth.blurred_noise((1, 500, 500), sigma=4.0, porosity=0.6, seed=11)
    return synth.overlapping_spheres((1, 500, 500), r2=144, porosity=0.6, seed=12)


@pytest.mark.parametrize("kind", ["noise", "disks"])
def test_decomposition_of_the_disagreement(kind):
    img = _image(kind)
    inl = synth.face_mask(img.shape, axis=1, index=0)
    rows, n_pore = _levels(img, inl)
    for r in rows:
        assert r["mio_in_conf"], r                      # the envelope holds the opening
        assert r["eq_in_conf"], r                       # equal count is reached before the next pressure
        assert r["b"] == r["a"] + r["gap"], r           # the two sides of the difference
        assert r["dis"] == 2 * r["a"] + r["gap"], r     # equals the comparison's count
        assert r["a"] <= r["excess"], r                 # larger balls within the envelope's excess
        assert r["gap"] >= 0 and (r["next_step"] == 0 or r["gap"] < r["next_step"]), r
        assert r["a"] <= 0.005 * n_pore, r              # the lattice part stays below 0.5 %
    # the smallest ball (one voxel) ends both methods on the reachable pore
    assert rows[-1]["T"] == 1 and rows[-1]["dis"] == 0


def test_lattice_part_falls_with_resolution():
    """One disk geometry rendered at 1 and 2 pixels per unit: the largest a
    and the largest envelope excess, as fractions of the pore pixels, fall
    (25 levels at the same physical radii)."""
    out = []
    for scale in (1, 2):
        img = synth.poisson_disks(L=250, r=12.0, porosity=0.6, seed=12, scale=scale)
        inl = synth.face_mask(img.shape, axis=1, index=0)
        rmax = np.sqrt(float(oracle.edt(img).max())) / scale
        T = sorted({max(1, int(np.ceil((scale * rmax * i / 25) ** 2))) for i in range(1, 26)}, reverse=True)
        rows, n_pore = _levels(img, inl, T)
        for r in rows:
            assert r["mio_in_conf"] and r["b"] == r["a"] + r["gap"], r
        out.append((max(r["a"] for r in rows) / n_pore, max(r["excess"] for r in rows) / n_pore))
    (a1, e1), (a2, e2) = out
    assert a2 < 0.8 * a1, out
    assert e2 < 0.8 * e1, out
