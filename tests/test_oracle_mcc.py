"""Pins of the oracle's null-collision Monte Carlo (Sec. 2.1, null-collision
method with a per-particle counter-based generator) and of the generator."""
import math

import numpy as np
import pytest
from scipy import stats

import ecpic_inputs as E
from ecpic_inputs import EPS0, KB, M_AR, ME, MU0, QE


def test_philox_matches_numpy_bit_for_bit(og):
    # numpy's Philox bit generator is Philox4x64-10; it increments its counter
    # before producing the first block.
    rng = np.random.default_rng(5)
    for _ in range(40):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        bg = np.random.Philox(counter=ctr, key=key)
        ref = [int(x) for x in bg.random_raw(4)]
        ours = og.philox4x64_10([ctr[0] + 1, ctr[1], ctr[2], ctr[3]], key)
        assert ours == ref


def test_child_uid_is_splitmix64_finaliser(og):
    # SplitMix64 from state 0: first output 0xE220A8397B1DCDAF (top bit set)
    assert og.child_uid(0, 0) == 0xE220A8397B1DCDAF
    uids = {og.child_uid(p, s) for p in range(200) for s in range(50)}
    assert len(uids) == 200 * 50 and all(u >> 63 for u in uids)


def test_cross_sections_and_bound(og):
    el, ex, iz = og.cross_sections(5.0)
    assert el == 1e-19 and ex == 0 and iz == 0
    el, ex, iz = og.cross_sections(15.76 * math.e)
    assert ex == pytest.approx(1e-20 * (1 - 11.5 / (15.76 * math.e)))
    assert iz == pytest.approx(8e-20 / math.e)  # ln(x)/x at x = e
    mcc = dict(n_gas=1e21, T_gas=300.0, m_gas=M_AR, eps_max_ev=1000.0, seed=1)
    numax = og.nu_max(mcc, 1, ME)
    for e in np.geomspace(1e-3, 1000.0, 4001):
        s = sum(og.cross_sections(e))
        assert 1e21 * s * math.sqrt(2 * e * QE / ME) <= numax
    assert og.nu_max(mcc, 2, M_AR) == pytest.approx(1.05 * 1e21 * 5e-19 * math.sqrt(2000 * QE / M_AR))


def _mono_electrons(og, n, e_ev, seed=3):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0)
    v = math.sqrt(2 * e_ev * QE / ME)
    return og.Species(-QE, ME, 10.0, rng.random(n) * 8, rng.random(n) * 8, v * d[0], v * d[1],
                      v * d[2], np.arange(n, dtype=np.uint64), cap=3 * n)


def test_electron_process_counts_and_energy_bookkeeping(og):
    n, e0 = 200_000, 40.0
    g = og.Grid(8, 8, 0.01, 0.01, 2.0, 1e-10, EPS0, MU0)
    el = _mono_electrons(og, n, e0)
    ions = og.Species(QE, M_AR, 10.0, [], [], [], [], [], np.zeros(0, np.uint64), cap=n)
    mcc = dict(n_gas=2e21, T_gas=300.0, m_gas=M_AR, eps_max_ev=1000.0, seed=9,
               electron_sid=0, ion_sid=1)
    ke0 = 0.5 * ME * 10.0 * np.sum(el.vr[:n] ** 2 + el.vt[:n] ** 2 + el.vz[:n] ** 2)
    d = og.Grid.collide(g, [el, ions], mcc, step=17)
    assert d["rc"] == 0
    numax = og.nu_max(mcc, 1, ME)
    pnull = 1 - math.exp(-numax * g.dt)
    v = math.sqrt(2 * e0 * QE / ME)
    sel, sex, siz = og.cross_sections(e0)
    p = np.array([sel, sex, siz]) * 2e21 * v / numax * pnull
    p = np.append(p, 1 - p.sum())
    # classify by the post-collision energy of the first n electrons
    e1 = 0.5 * ME * (el.vr[:n] ** 2 + el.vt[:n] ** 2 + el.vz[:n] ** 2) / QE
    n_iz = d["n_ionized"]
    n_ex = int(np.sum(np.abs(e1 - (e0 - 11.5)) < 1e-9))
    n_el = int(np.sum((np.abs(e1 - e0) > 1e-12) & (np.abs(e1 - e0) < 0.01)))
    obs = np.array([n_el, n_ex, n_iz, n - n_el - n_ex - n_iz])
    assert obs[:3].min() > 100
    chi2 = np.sum((obs - n * p) ** 2 / (n * p))
    assert stats.chi2.sf(chi2, 3) > 1e-3
    # pairs created at the parent's position, charge-neutral
    assert el.n == n + n_iz and ions.n == n_iz
    assert np.array_equal(el.xi[n:el.n], ions.xi[:n_iz])
    # exact energy bookkeeping: initial = final (all species) + collisional loss
    ke1 = sum(0.5 * s.m * s.w * np.sum(s.vr[: s.n] ** 2 + s.vt[: s.n] ** 2 + s.vz[: s.n] ** 2)
              for s in (el, ions))
    assert ke0 - ke1 == pytest.approx(d["w_coll"], rel=1e-12)
    # isotropic scattering: mean direction of collided electrons ~ 0
    hit = np.abs(e1 - e0) > 1e-12
    vv = np.stack([el.vr[:n][hit], el.vt[:n][hit], el.vz[:n][hit]])
    dirs = vv / np.linalg.norm(vv, axis=0)
    assert np.abs(dirs.mean(axis=1)).max() < 5 / math.sqrt(hit.sum())
    # determinism: same seed and step give the same outcome
    el2 = _mono_electrons(og, n, e0)
    ions2 = og.Species(QE, M_AR, 10.0, [], [], [], [], [], np.zeros(0, np.uint64), cap=n)
    og.Grid.collide(g, [el2, ions2], mcc, step=17)
    assert np.array_equal(el.vr[: el.n], el2.vr[: el2.n])


def test_ion_charge_exchange_rate(og):
    # cold ions in a 300 K gas: mean relative speed is the gas mean speed
    n = 200_000
    g = og.Grid(8, 8, 0.01, 0.01, 2.0, 1e-8, EPS0, MU0)
    rng = np.random.default_rng(4)
    ions = og.Species(QE, M_AR, 1.0, rng.random(n) * 8, rng.random(n) * 8, np.zeros(n),
                      np.zeros(n), np.zeros(n), np.arange(n, dtype=np.uint64))
    el = og.Species(-QE, ME, 1.0, [], [], [], [], [], np.zeros(0, np.uint64), cap=1)
    mcc = dict(n_gas=1e21, T_gas=300.0, m_gas=M_AR, eps_max_ev=1.0, seed=2,
               electron_sid=0, ion_sid=1)
    d = og.Grid.collide(g, [el, ions], mcc, step=3)
    numax = og.nu_max(mcc, 2, M_AR)
    pnull = 1 - math.exp(-numax * g.dt)
    gbar = math.sqrt(8 * KB * 300.0 / (math.pi * M_AR))
    p = pnull * 1e21 * 5e-19 * gbar / numax
    k = d["n_coll"][1]
    assert abs(k - n * p) < 5 * math.sqrt(n * p * (1 - p))
    hit = ions.vr[:n] != 0
    # exchanged ions carry neutrals drawn from the gas Maxwellian weighted by
    # the relative speed |v_n| (rate ~ g): <v_r^2> = E|v|^3 / (3 E|v|) = 4kT/(3M)
    assert np.mean(ions.vr[:n][hit] ** 2) == pytest.approx(4 * KB * 300 / (3 * M_AR), rel=0.03)
    assert hit.sum() == k
