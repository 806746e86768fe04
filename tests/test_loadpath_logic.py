"""Host logic of the adaptive load path (loadpath.solve) on the CPU, with the
library calls replaced by stand-ins: increment growth and cutback, the exact
end point, the lower limit of the increment, the extrapolated Newton start
and the prescribed values on the constrained dofs, the convergence target."""
import types

import pytest

torch = pytest.importorskip("torch")

from paper_2606_17390_amd import fem, loadpath  # noqa: E402


class Env:
    """Stand-ins for the library; fail(t, dt) -> True makes an increment fail."""

    def __init__(self, monkeypatch, fail=lambda t, dt: False, its=2, reaction=5.0):
        self.calls = []
        self.fail = fail
        self.its = its
        n = 4
        self.mesh = types.SimpleNamespace(n_nodes=n)
        self.params = types.SimpleNamespace(model=0)
        self.bc = torch.zeros(3 * n, dtype=torch.uint8)
        self.bc[:3] = 1  # node 0 constrained
        self.u1 = torch.arange(1.0, 3 * n + 1, dtype=torch.float64).reshape(n, 3)
        self.t = 0.0
        self.pred = []  # (d, hist) of the tangent-start evaluations
        out = types.SimpleNamespace(K=None, R=torch.zeros(3 * n, dtype=torch.float64))
        monkeypatch.setattr(fem, "Forward", lambda *a, **k: out)
        monkeypatch.setattr(fem, "residual_tangent",
                            lambda m, c, p, d, h, **k: self.pred.append((d.clone(), k)) or out)
        solver = types.SimpleNamespace(solve=lambda K, b, **k: (torch.zeros_like(b), 3, 1e-5))
        # (the stand-in product returns zeros, so the tangent start's right-hand side is -R_n = 0)
        monkeypatch.setattr(fem, "Solver", lambda *a, **k: solver)
        monkeypatch.setattr(fem, "csr_spmv", lambda csr, K, x: self.spmv.append(x.clone()) or torch.zeros_like(x))
        self.spmv = []
        monkeypatch.setattr(loadpath, "reaction_norm", lambda *a, **k: reaction)
        monkeypatch.setattr(loadpath.newton, "solve_step", self.solve_step)

    def solve_step(self, mesh, csr, params, d, hist, bc_mask, **kw):
        dt = float(d[0, 0]) / float(self.u1[0, 0]) - self.t  # prescribed value of dof 0 is (t + dt) u1
        self.calls.append(dict(t=self.t, dt=dt, d=d.clone(), kw=kw))
        if self.fail(self.t, dt):
            raise RuntimeError("no convergence")
        # the "solution": free dofs set to a smooth function of the load factor
        tn = self.t + dt
        free = ~bc_mask.bool().view(-1)
        d.view(-1)[free] = (tn + tn * tn) * self.u1.view(-1)[free]
        self.t = tn
        kw["trace"].append((10, 1e-3, 1.0, 0.0, 1e-2))
        return hist + 1.0, self.its, [1.0, 1e-9]

    def run(self, **kw):
        return loadpath.solve(self.mesh, None, self.params, self.bc, self.u1, torch.zeros(7, 8), **kw)


def test_growth_and_exact_end(monkeypatch):
    env = Env(monkeypatch)
    res = env.run(dt0=1e-3, dt_max=5e-2)
    dts = [s[1] for s in res["steps"]]
    # 1e-3 doubling to the cap, then the cap, the last one clipped to end at t = 1
    assert dts[:6] == pytest.approx([1e-3, 2e-3, 4e-3, 8e-3, 1.6e-2, 3.2e-2])
    assert all(x == pytest.approx(5e-2) for x in dts[6:-1]) and dts[-1] <= 5e-2
    assert res["steps"][-1][0] == pytest.approx(1.0, abs=1e-12) and sum(dts) == pytest.approx(1.0)
    # 10 per Newton trace entry, 3 for the tangent start of the first increment
    assert res["newton_iterations"] == 2 * len(dts) and res["linear_iterations"] == 10 * len(dts) + 3
    assert not res["failed"]
    assert float(res["hist"][0, 0]) == len(dts)  # every accepted increment commits its history


def test_cutback_and_recovery(monkeypatch):
    # increments larger than 2.5e-3 fail before t = 0.01
    env = Env(monkeypatch, fail=lambda t, dt: t < 0.01 and dt > 2.5e-3)
    res = env.run(dt0=1e-3, dt_max=5e-2, t_end=0.05)
    assert res["failed"] and all(f[1] > 2.5e-3 for f in res["failed"])
    assert all(s[1] <= 2.5e-3 + 1e-15 for s in res["steps"] if s[0] <= 0.01)
    assert res["steps"][-1][0] == pytest.approx(0.05, abs=1e-12)
    # a failure halves the increment, which then grows again
    f0 = env.calls.index(next(c for c in env.calls if c["dt"] > 2.5e-3))
    assert env.calls[f0 + 1]["dt"] == pytest.approx(env.calls[f0]["dt"] / 2)


def test_increment_below_minimum_raises(monkeypatch):
    env = Env(monkeypatch, fail=lambda t, dt: True)
    with pytest.raises(RuntimeError, match="increment below"):
        env.run(dt0=1e-3, dt_min=1e-5)
    dts = [c["dt"] for c in env.calls]
    assert dts[0] == pytest.approx(1e-3) and dts[-1] >= 1e-5 > dts[-1] / 2
    assert len(dts) == 7  # 1e-3 / 2^k for k = 0..6 (1.5625e-5); the next would be below 1e-5


def test_extrapolated_start_and_prescribed_values(monkeypatch):
    env = Env(monkeypatch)
    env.run(dt0=1e-3, dt_max=5e-2, t_end=0.02)
    bc = env.bc.bool().view(-1)
    c = env.calls
    # first increment: previous solution (zero) with the prescribed values
    assert torch.equal(c[0]["d"].view(-1)[~bc], torch.zeros(int((~bc).sum()), dtype=torch.float64))
    assert c[0]["kw"]["eta0"] is None  # the tangent start took the first_eta solve
    # tangent start: K and R at the converged state (zero), K applied to the boundary increment
    assert len(env.pred) == 1 and not env.pred[0][0].any() and len(env.spmv) == 1
    assert torch.equal(env.spmv[0], c[0]["d"].view(-1))
    for k in range(2, len(c)):
        t0, t1 = c[k - 2]["t"] + c[k - 2]["dt"], c[k - 1]["t"] + c[k - 1]["dt"]
        f = lambda t: t + t * t  # noqa: E731  (the stand-in solution's profile)
        pred = f(t1) + (c[k]["dt"] / c[k - 1]["dt"]) * (f(t1) - f(t0))
        d = c[k]["d"].view(-1)
        assert torch.allclose(d[~bc], pred * env.u1.view(-1)[~bc], rtol=1e-14)
        assert torch.allclose(d[bc], (c[k]["t"] + c[k]["dt"]) * env.u1.view(-1)[bc], rtol=1e-14)
        assert c[k]["kw"]["eta0"] is None


def test_without_tangent_start_the_first_solve_is_tight(monkeypatch):
    env = Env(monkeypatch)
    res = env.run(dt0=1e-3, t_end=3e-3, tangent_start=False)
    assert not env.pred and env.calls[0]["kw"]["eta0"] == 1e-4 and env.calls[1]["kw"]["eta0"] is None
    assert res["linear_iterations"] == 10 * len(res["steps"])


def test_convergence_target_follows_the_reaction(monkeypatch):
    env = Env(monkeypatch, reaction=8.0)
    env.run(dt0=1e-3, t_end=3e-3, ftol=1e-6)
    c = env.calls
    # before any reaction: relative to the first residual; afterwards 1e-6 of the reaction norm
    assert c[0]["kw"]["tol"] == 1e-6 and c[0]["kw"]["atol"] == 0.0
    assert c[1]["kw"]["tol"] == 0.0 and c[1]["kw"]["atol"] == pytest.approx(8e-6)
