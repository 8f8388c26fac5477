"""Training entry points on the GPU, through the C ABI: the two loss forms
against the oracle (the per-atom mean and Eq. 7's half sum), the host-pointer
loss gradient, parameters set from device memory, the device Adam step, and
the torch.autograd.Function around the hand-written weight gradient."""
import numpy as np
import pytest

from paper_2107_11311_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_2107_11311_amd import aenet
    aenet.load()
    return aenet


@pytest.fixture(scope="module")
def batch(orc):
    """Three water boxes of unequal size (64, 70 and 81 molecules: the two loss
    forms weight them differently) with references from a second network."""
    m = I.load_model("water4096")
    ref = I.load_model("water4096_ref")
    boxes = [I.water_box(k, 3100 + k) for k in (64, 70, 81)]
    offs = np.cumsum([0] + [len(b.pos) for b in boxes]).astype(np.int64)
    pos = np.vstack([b.pos for b in boxes])
    sp = np.concatenate([b.species for b in boxes]).astype(np.int32)
    bx = np.vstack([b.box for b in boxes])
    er, fr = [], []
    for b in boxes:
        E, _, F = orc.energy_forces(ref, b.pos, b.species, b.box, b.pbc)
        er.append(E)
        fr.append(F)
    return m, offs, pos, sp, bx, np.array(er), np.vstack(fr)


def _dev_loss_grad(A, ctx, offs, pos, sp, bx, er, fr, lam):
    import torch
    dev = torch.device("cuda:0")
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    grad = torch.zeros(ctx.n_params(), dtype=torch.float64, device=dev)
    ctx.loss_grad_dev(offs, torch.from_numpy(pos).to(dev), sp, bx, (1, 1, 1), torch.from_numpy(er).to(dev),
                      torch.from_numpy(fr).to(dev), lam, loss, grad)
    torch.cuda.synchronize()
    return loss.item(), grad.cpu().numpy()


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_loss_forms_match_oracle(A, orc, batch, form, lam):
    m, offs, pos, sp, bx, er, fr = batch
    ctx = A.Context(m, "fp64")
    ctx.set_loss_form(form)
    L, g = _dev_loss_grad(A, ctx, offs, pos, sp, bx, er, fr, lam)
    L0, g0 = orc.loss_grad(m, offs, pos, sp, bx, (1, 1, 1), er, fr, lam, form=form)
    print(f"form {form} lambda {lam}: loss {L:.12e} oracle {L0:.12e}")
    assert abs(L - L0) <= 1e-10 * abs(L0)
    assert np.abs(g - g0).max() <= 1e-9 * np.abs(g0).max()
    # the host-pointer entry point is the same computation
    Lh, gh = ctx.loss_grad(offs, pos, sp, bx, (1, 1, 1), er, fr, lam)
    assert Lh == L and np.array_equal(gh, g)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_set_params_dev_equals_host(A, precision):
    import torch
    m = I.load_model("water64")
    s = I.make_system("water64")
    p = m.flat_params() * (1.0 + 0.05 * np.random.default_rng(9).normal(size=m.n_params()))
    host = A.Context(m, precision)
    devc = A.Context(m, precision)
    host.set_params(p)
    devc.set_params_dev(torch.from_numpy(p).to("cuda:0"))
    r1 = host.energy_forces(s.pos, s.species, s.box, s.pbc)
    r2 = devc.energy_forces(s.pos, s.species, s.box, s.pbc)
    assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])
    assert np.array_equal(devc.get_params(), p)
    # non-finite values are refused and leave the parameters as they were
    bad = torch.from_numpy(p).to("cuda:0")
    bad[7] = float("nan")
    with pytest.raises(A.AenetError) as e:
        devc.set_params_dev(bad)
    assert e.value.code == A.AENET_E_NONFINITE
    assert np.array_equal(devc.get_params(), p)
    host.close()
    devc.close()


def test_adam_step_dev(A):
    """Three Adam steps on the device against the update rule of Kingma and
    Ba (2015) written out here in numpy."""
    import torch
    g = np.random.default_rng(4)
    n = 1001
    p, m, v = g.normal(size=n), np.zeros(n), np.zeros(n)
    tp, tm, tv = (torch.from_numpy(x.copy()).to("cuda:0") for x in (p, m, v))
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for t in range(1, 4):
        gr = g.normal(size=n)
        A.adam_step_dev(tp, torch.from_numpy(gr).to("cuda:0"), tm, tv, lr, b1, b2, eps, t)
        m = b1 * m + (1 - b1) * gr
        v = b2 * v + (1 - b2) * gr * gr
        p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    torch.cuda.synchronize()
    np.testing.assert_allclose(tp.cpu().numpy(), p, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(tm.cpu().numpy(), m, rtol=1e-14, atol=1e-16)


def test_autograd_function_gradient(A, orc, batch):
    """loss.backward() through the torch.autograd.Function gives the
    oracle's parameter gradient and central finite differences of the cost."""
    import torch
    from paper_2107_11311_amd.autograd import Batch, energy_force_loss
    m, offs, pos, sp, bx, er, fr = batch
    dev = torch.device("cuda:0")
    ctx = A.Context(m, "fp64")
    b = Batch(offs, torch.from_numpy(pos).to(dev), sp, bx, np.ones(3, np.uint8), torch.from_numpy(er).to(dev),
              torch.from_numpy(fr).to(dev), 1.0)
    p0 = m.flat_params()
    params = torch.nn.Parameter(torch.from_numpy(p0.copy()).to(dev))
    loss = energy_force_loss(params, ctx, b)
    (3.0 * loss).backward()           # the incoming gradient is applied
    g = params.grad.cpu().numpy() / 3.0
    L0, g0 = orc.loss_grad(m, offs, pos, sp, bx, (1, 1, 1), er, fr, 1.0)
    assert abs(loss.item() - L0) <= 1e-10 * abs(L0)
    assert np.abs(g - g0).max() <= 1e-9 * np.abs(g0).max()
    h = 1e-5
    idx = list(np.random.default_rng(5).choice(len(p0), 12, replace=False)) + [len(p0) - 1]
    with torch.no_grad():
        for k in idx:
            pp = torch.from_numpy(p0.copy()).to(dev)
            pp[k] += h
            lp = energy_force_loss(pp, ctx, b).item()
            pp[k] -= 2 * h
            lm = energy_force_loss(pp, ctx, b).item()
            fd = (lp - lm) / (2 * h)
            assert abs(g[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (k, g[k], fd)
    ctx.close()
