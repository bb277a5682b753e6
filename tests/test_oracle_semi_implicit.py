"""Pin of the oracle's semi-implicit transport (section "Semi-implicit Euler-Maruyama
method", eqs. poisson_simp and conductivity, final algorithm steps 1-5) by a two-layer
closed form: a neutral plasma in the lower half of a plane gap, D = 0.  After one
transport the field must be the layered dielectric solution with eps_l = 1 + sigma dt /
eps0, sigma = e mu(V/L) n, and every electron must have moved by -mu(|E^k|) E^{k+1} dt.
Dropping sigma, advecting with E^k, or taking the mobility at E^{k+1} each fail here."""
import numpy as np
import pytest

from paper_2307_01797_amd import workloads

from semi_implicit_case import ez_column, make_case


@pytest.mark.parametrize("eps_jump", [0.5, 3.0])
def test_two_layer_conductivity_closed_form(orc, eps_jump):
    base = workloads.preset("streamer_64")
    c = make_case(base, eps_jump=eps_jump)
    cfg, grid = c["cfg"], c["cfg"]["grid"]
    sim = orc.Sim(cfg)
    sim.set_particles(c["xi"], c["w"], c["ids"])
    sim.set_counts("plus", c["nplus"])
    sim.transport(cfg["dt"])
    phi, Ex, Ey, Ez = sim.field()
    E_h = c["E_h"]
    # the step's field: layered solution, uniform over each x-y plane, no x-y component
    col, spread = ez_column(Ez, grid)
    assert np.allclose(col, c["Ez_col"], rtol=1e-9, atol=0)
    assert spread.max() <= 1e-9 * E_h
    assert np.abs(Ex).max() <= 1e-9 * E_h and np.abs(Ey).max() <= 1e-9 * E_h
    # the layers really differ (eps_l E_l = E_h): the conductivity entered the solve
    assert c["E_h"] / c["E_l"] == pytest.approx(c["eps_l"], rel=1e-12)
    assert c["eps_l"] - 1.0 == pytest.approx(eps_jump, rel=1e-6)
    # advection with mu^k E^{k+1}(X^k) dt, no diffusion (D = 0)
    xi, w, ids = sim.particles()
    assert len(ids) == len(c["ids"])
    o = np.argsort(ids)
    p = np.argsort(c["ids"])
    assert np.array_equal(ids[o], c["ids"][p])
    d = xi[o] - c["xi"][p]
    assert np.abs(d[:, 0]).max() <= 1e-12 and np.abs(d[:, 1]).max() <= 1e-12
    assert np.allclose(d[:, 2], c["dz"][p], rtol=1e-9, atol=0)
    assert np.array_equal(w[o], c["w"][p])


def test_two_layer_mistakes_are_visible(orc):
    # the closed form separates the readings a wrong implementation would take
    c = make_case(workloads.preset("streamer_64"), eps_jump=1.0)
    V_L = c["cfg"]["V_anode"] / (c["cfg"]["grid"][2] * c["dx"])
    assert abs(c["E_l"] - V_L) > 0.3 * V_L          # sigma dropped: E_l would be V/L
    assert abs(c["E_h"] - c["E_l"]) > 0.5 * c["E_l"]  # E^k instead of E^{k+1}
    mu_b = c["cfg"]["coeffs"]["mu_b"]
    assert abs((c["E_l"] / V_L) ** mu_b - 1.0) > 0.1  # mobility at E^{k+1} instead of E^k


def test_residual_and_field_push_entries_reproduce_transport(orc):
    """The oracle entries that check GPU states at full size: the residual of the
    oracle's own solution in the system rebuilt from the pre-transport state is at the
    solver's tolerance (and a perturbed potential is not), and the push with the two
    given fields reproduces the transport's positions bit for bit."""
    cfg = workloads.preset("streamer_64", grid=(16, 16, 16), dx=1e-3 / 64,
                           seed_centre=(125e-6, 125e-6, 125e-6), seed_sigma=30e-6,
                           V_anode=18e3 * 0.25)
    a = orc.Sim(cfg)
    a.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    a.step(cfg["dt"], 3)
    xi, w, ids = a.particles()
    counts = {k: a.counts(k) for k in ("plus", "minus", "gamma")}
    phi_k, ex, ey, ez = a.field()
    step = a.diagnostics()["step"]
    b = orc.Sim(cfg)
    b.set_particles(xi, w, ids)
    for k, v in counts.items():
        b.set_counts(k, v)
    b.set_field(phi_k)
    b.set_step(step)
    a.transport(cfg["dt"])
    phi1, e1x, e1y, e1z = a.field()
    assert b.semi_implicit_residual(cfg["dt"], phi1) < 1e-12
    bad = phi1.copy()
    bad[len(bad) // 2] *= 1.0 + 1e-6
    assert b.semi_implicit_residual(cfg["dt"], bad) > 1e-8
    assert b.semi_implicit_residual(cfg["dt"], phi_k) > 1e-6   # the old potential
    x1 = orc.push_with_fields(cfg, xi, ids, step, cfg["dt"], (ex, ey, ez), (e1x, e1y, e1z))
    xa, _, ida = a.particles()
    o1, o2 = np.argsort(ids), np.argsort(ida)
    inside = np.all((x1[o1] >= 0) & (x1[o1] < 16), axis=1)
    assert np.array_equal(ids[o1][inside], ida[o2])
    assert np.array_equal(x1[o1][inside], xa[o2])
