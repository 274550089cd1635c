"""The stored config-1 fixture (tests/golden/, written by make_golden.py from
the oracle alone) still matches the oracle, and is close to Chang-Lundgren.

The fixture guards against unnoticed changes of the oracle's arithmetic; any
intended change must regenerate it in a commit that names the passage of the
paper (or the reading of it) that justifies the change.
"""
import json
import os

import numpy as np

import oracle
from oracle import derive

GOLD = os.path.join(os.path.dirname(__file__), "golden", "config1_hartmann_link.json")


def test_config1_fixture_matches_oracle(orc):
    g = json.load(open(GOLD))
    p = derive.hartmann_params(8, 64, oracle.LINK, 0.8, 0.8, 10.0, 0.1, 0.05)
    assert abs(p.b0 - g["params"]["b0"]) < 1e-18 and abs(p.fx - g["params"]["fx"]) < 1e-20
    s = orc.init_state(p)
    orc.run(p, s, 20000, nthreads=2)
    o = orc.observe(p, s)
    assert np.abs(o["ux"][:, 0] - np.array(g["ux"])).max() < 1e-15
    assert np.abs(o["bx"][:, 0] - np.array(g["bx"])).max() < 1e-15
    # all columns identical (x-invariant run)
    assert np.array_equal(o["ux"], np.repeat(o["ux"][:, :1], 8, axis=1))


def test_config1_close_to_chang_lundgren():
    g = json.load(open(GOLD))
    u = np.array(g["ux"]) / g["u_ref"]
    b = np.array(g["bx"]) / g["b_ref"]
    ua, ba = np.array(g["chang_lundgren_u_star"]), np.array(g["chang_lundgren_b_star"])
    # 20000 steps from rest at a = 32 is close to, not at, the steady state
    assert np.sqrt(np.mean((u - ua) ** 2)) / np.abs(ua).max() < 2e-2
    assert np.sqrt(np.mean((b - ba) ** 2)) / np.abs(ba).max() < 2e-2


PREC = os.path.join(os.path.dirname(__file__), "golden", "precision_case_512.json")


def test_precision_case_fixture_matches_oracle(orc):
    """512-row precision case (Ha = 50, c = 0.5): the stored 20 000-step
    columns are what the oracle computes now."""
    g = json.load(open(PREC))
    p = derive.hartmann_params(1, 512, oracle.LINK, 0.8, 0.8, 50.0, 0.5, 0.003)
    assert p.b0 == g["params"]["b0"] and p.fx == g["params"]["fx"]
    s = orc.init_state(p)
    orc.run(p, s, 20000, nthreads=4)
    o = orc.observe(p, s)
    assert np.array_equal(o["ux"][:, 0], np.array(g["ux_20000"]))
    assert np.array_equal(o["bx"][:, 0], np.array(g["bx_20000"]))


def test_precision_case_steady_state_is_chang_lundgren():
    """The stored steady state agrees with the closed form (Sec. VIII's
    Chang-Lundgren profile) to the discretisation error at a = 256, Ha = 50
    (second order: of order (Ha / a)^2 / 10 relative), and is symmetric."""
    g = json.load(open(PREC))
    assert g["steady_residual"] < 1e-12
    u = np.array(g["ux_steady"]) / g["u_ref"]
    b = np.array(g["bx_steady"]) / g["b_ref"]
    ua, ba = np.array(g["chang_lundgren_u_star"]), np.array(g["chang_lundgren_b_star"])
    assert np.sqrt(np.mean((u - ua) ** 2)) / np.sqrt(np.mean(ua ** 2)) < 2e-3
    assert np.sqrt(np.mean((b - ba) ** 2)) / np.sqrt(np.mean(ba ** 2)) < 2e-3
    assert np.abs(u - u[::-1]).max() < 1e-9 * np.abs(u).max()
    assert np.abs(b + b[::-1]).max() < 1e-9 * np.abs(b).max()


COUETTE = os.path.join(os.path.dirname(__file__), "golden", "couette_256_link_1000.json")


def test_couette256_fixture_matches_oracle(orc):
    """The stored 256-row Hartmann-Couette columns (benchmark workload,
    1000 steps from rest) are what the oracle computes now."""
    g = json.load(open(COUETTE))
    p = derive.couette_params(4, 256, oracle.LINK, 0.7, 0.9, 50.0, 1.0, 1.0, 0.05)
    assert p.b0 == g["params"]["b0"]
    s = orc.init_state(p)
    orc.run(p, s, 1000, nthreads=4)
    o = orc.observe(p, s)
    assert np.array_equal(o["ux"][:, 0], np.array(g["ux"]))
    assert np.array_equal(o["bx"][:, 0], np.array(g["bx"]))


def test_duct_far_from_its_side_walls_is_the_channel():
    """The stored 256 x 256 duct (3D oracle) at its mid layer against the
    stored 256-row channel (2D oracle), both 1000 steps from rest.  Side-wall
    effects reach the mid layer in that time only acoustically (sound at
    c_s = 0.58 nodes per step crosses 128 layers; diffusion and Alfven waves
    do not), which leaves a few 1e-5; the layers near the wall differ at
    order one."""
    here = os.path.join(os.path.dirname(__file__), "golden")
    duct = json.load(open(os.path.join(here, "duct_256_link_1000.json")))
    chan = json.load(open(os.path.join(here, "couette_256_link_1000.json")))
    for k in ("ux", "bx"):
        ref = np.asarray(chan[k])
        rows = dict(zip(duct["layers"], (np.asarray(r) for r in duct[k])))
        assert np.linalg.norm(rows[128] - ref) / np.linalg.norm(ref) < 1e-4
        assert np.linalg.norm(rows[0] - ref) / np.linalg.norm(ref) > 0.1


def test_cavity_fixture_is_an_enclosure_flow():
    """The stored cavity: the lid drags the top layer along +x, a return flow
    runs along -x below it, and u_y changes sign across the cavity (the
    recirculation); the field is induced (B_x non-zero)."""
    here = os.path.join(os.path.dirname(__file__), "golden")
    g = json.load(open(os.path.join(here, "cavity_512_link_1000.json")))
    ux, uy, bx = (np.asarray(g[k]) for k in ("ux", "uy", "bx"))
    assert ux[-1].mean() > 0.01 and ux[:-1].min() < 0
    assert uy.max() > 0 > uy.min()
    assert np.abs(bx).max() > 0
