"""torch.autograd wrappers: the library's adjoints against finite differences and the oracle."""
import numpy as np
import pytest
import torch

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2402_18311_amd import autograd, hybro
    nl = netgen.make_small(300, 320, 16, seed=9, n_fixed=6)
    pl = hybro.Placer(nl, precision=64)
    obj = autograd.PlacementObjective(pl, 4 * nl.bin_w, grad_mode=1)
    return nl, pl, obj


def _xy(nl, seed):
    x, y = nl.random_positions(seed)
    dev = torch.device("cuda")
    return (torch.tensor(x, dtype=torch.float64, device=dev, requires_grad=True),
            torch.tensor(y, dtype=torch.float64, device=dev, requires_grad=True))


def test_wirelength_gradcheck(setup):
    """The WA adjoint (per-pin gradients of Eq. 3 reduced to cells) is the derivative of the
    library's own wirelength: torch.autograd.gradcheck with central differences."""
    nl, pl, obj = setup
    x, y = _xy(nl, 1)
    assert torch.autograd.gradcheck(lambda a, b: obj.wirelength(a, b), (x, y), eps=1e-6,
                                    atol=1e-6, rtol=1e-5)


def test_density_adjoint_matches_oracle_and_fd(setup, orc):
    """The exact density adjoint equals the oracle's (same definition, FP64), and matches central
    differences of the oracle's continuous-map energy up to the 2^-12 quantisation of the
    charge rectangles in the map that psi comes from."""
    nl, pl, obj = setup
    x, y = _xy(nl, 2)
    n = obj.density_energy(x, y)
    n.backward()
    g = np.concatenate([x.grad.cpu().numpy(), y.grad.cpu().numpy()])
    o = orc.Oracle(nl)
    xs, ys = x.detach().cpu().numpy(), y.detach().cpu().numpy()
    ref = o.eval(xs, ys, 4 * nl.bin_w, grad_mode=1)
    assert float(n) == pytest.approx(ref["energy"], rel=1e-10)
    gref = np.concatenate([ref["gdx"], ref["gdy"]])
    assert np.linalg.norm(g - gref) / np.linalg.norm(gref) < 1e-9
    h = 1e-6
    fd = np.zeros_like(g)
    idx = np.random.default_rng(0).choice(len(xs), 40, replace=False)
    for i in idx:
        for ax, arr in ((0, xs), (1, ys)):
            a = arr.copy()
            a[i] += h
            ep = o.energy_float(a, ys) if ax == 0 else o.energy_float(xs, a)
            a[i] -= 2 * h
            em = o.energy_float(a, ys) if ax == 0 else o.energy_float(xs, a)
            fd[ax * len(xs) + i] = (ep - em) / (2 * h)
    sel = np.concatenate([idx, idx + len(xs)])
    assert np.linalg.norm(g[sel] - fd[sel]) / np.linalg.norm(fd[sel]) < 2e-3


def test_objective_is_wirelength_plus_lambda_energy(setup):
    nl, pl, obj = setup
    lam = 0.3
    x, y = _xy(nl, 3)
    f = obj.objective(x, y, lam)
    f.backward()
    gf = torch.cat([x.grad, y.grad]).clone()
    x.grad = None
    y.grad = None
    w = obj.wirelength(x, y)
    d = obj.density_energy(x, y)
    (w + lam * d).backward()
    g2 = torch.cat([x.grad, y.grad])
    assert float(f) == pytest.approx(float(w) + lam * float(d), rel=1e-12)
    assert torch.linalg.norm(gf - g2) / torch.linalg.norm(gf) < 1e-10


@pytest.mark.parametrize("prec,grad_mode", [(32, 1), (32, 0), (64, 0)])
def test_density_only_evaluation_matches_oracle(orc, prec, grad_mode):
    """One density-only evaluation (no net sweep) gives lambda * grad N: the oracle's density
    gradient (exact adjoint or field force) to the parity bar, with wirelength 0, in FP32 too,
    where the former difference of two full evaluations cancelled."""
    from paper_2402_18311_amd import hybro
    nl = netgen.make_small(20_011, 21_003, 128, seed=3, n_fixed=40)
    pl = hybro.Placer(nl, precision=prec)
    s = pl.new_slot()
    x, y = nl.random_positions(4)
    pl.set_positions(s, x, y)
    px, py = pl.positions(s)
    lam = 0.7
    (wl, en, ov), gx, gy = pl.eval(s, 4 * nl.bin_w, lam=lam, grads=True,
                                   grad_mode=grad_mode | hybro.HP_GRAD_DENSITY_ONLY)
    o = orc.Oracle(nl)
    ref = o.eval(px.astype(np.float64), py.astype(np.float64), 4 * nl.bin_w, grad_mode=grad_mode)
    g = np.concatenate([gx.cpu().numpy()[0], gy.cpu().numpy()[0]]).astype(np.float64)
    gref = lam * np.concatenate([ref["gdx"], ref["gdy"]])
    tol = 1e-4 if prec == 32 else 1e-10
    assert wl[0] == 0.0
    assert en[0] == pytest.approx(ref["energy"], rel=1e-5 if prec == 32 else 1e-10)
    assert ov[0] == ref["overflow"]
    assert np.linalg.norm(g - gref) / np.linalg.norm(gref) < tol
    # a following full evaluation is unaffected (its sweep and totals are its own)
    (wl2, _, _), _, _ = pl.eval(s, 4 * nl.bin_w, lam=lam, grads=True, grad_mode=grad_mode)
    assert wl2[0] == pytest.approx(ref["wl"], rel=1e-5 if prec == 32 else 1e-10)
    with pytest.raises(hybro.HybroError):
        pl.eval(s, 4 * nl.bin_w, lam=-1.0, grad_mode=hybro.HP_GRAD_DENSITY_ONLY)
    pl.close()
