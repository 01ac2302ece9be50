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


def _speed2(s, lo, hi):
    return s.vr[lo:hi] ** 2 + s.vt[lo:hi] ** 2 + s.vz[lo:hi] ** 2


def test_elastic_recoil_matches_two_body_kinematics(og):
    # Below the excitation threshold every real collision is elastic.  For each
    # scattered electron the lab-frame angle is read off its velocities before
    # and after; momentum and energy conservation with a target at rest then
    # fix the speed ratio exactly:
    #   v'/v = (m cos t + sqrt(M^2 - m^2 sin^2 t)) / (m + M),
    # whose energy loss 1 - (v'/v)^2 = (2m/M)(1 - cos t) + O((m/M)^2).  A
    # recoil factor of m/M (or 4m/M) would be off by 50 % (or 100 %).
    n, e0 = 100_000, 5.0
    g = og.Grid(8, 8, 0.01, 0.01, 2.0, 1e-10, EPS0, MU0)
    el = _mono_electrons(og, n, e0, seed=11)
    v0 = np.stack([el.vr[:n].copy(), el.vt[:n].copy(), el.vz[:n].copy()])
    ions = og.Species(QE, M_AR, 10.0, [], [], [], [], [], np.zeros(0, np.uint64), cap=n)
    mcc = dict(n_gas=1e22, T_gas=300.0, m_gas=M_AR, eps_max_ev=100.0, seed=21,
               electron_sid=0, ion_sid=1)
    d = og.Grid.collide(g, [el, ions], mcc, step=4)
    assert d["rc"] == 0 and d["n_ionized"] == 0
    v1 = np.stack([el.vr[:n], el.vt[:n], el.vz[:n]])
    hit = np.any(v1 != v0, axis=0)
    assert hit.sum() == d["n_coll"][0] and hit.sum() > 5000
    a, b = v0[:, hit], v1[:, hit]
    sa, sb = np.linalg.norm(a, axis=0), np.linalg.norm(b, axis=0)
    cos_t = np.clip(np.sum(a * b, axis=0) / (sa * sb), -1.0, 1.0)
    m, M = ME, M_AR
    ratio = (m * cos_t + np.sqrt(M * M - m * m * (1 - cos_t ** 2))) / (m + M)
    loss_exact = 1 - ratio ** 2
    loss = 1 - (sb / sa) ** 2
    big = loss_exact > 1e-3 * 2 * m / M  # leave out grazing events (loss ~ roundoff)
    np.testing.assert_allclose(loss[big], loss_exact[big], rtol=1e-3)
    # isotropic scattering: <1 - cos t> = 1, so the mean loss is 2m/M
    k = hit.sum()
    assert np.mean(1 - cos_t) == pytest.approx(1.0, abs=5 * math.sqrt(1 / 3 / k))
    assert np.mean(loss) / (2 * m / M) == pytest.approx(1.0, abs=5 * math.sqrt(1 / 3 / k))
    assert ions.n == 0


def _ionising_run(og, n=200_000, e0=60.0, seed=13):
    g = og.Grid(8, 8, 0.01, 0.01, 2.0, 1e-10, EPS0, MU0)
    el = _mono_electrons(og, n, e0, seed=seed)
    # distinct positions identify a parent with the pair born at its place
    el.xi[:n] = np.arange(n) * (8.0 / n)
    ions = og.Species(QE, M_AR, 10.0, [], [], [], [], [], np.zeros(0, np.uint64), cap=n)
    mcc = dict(n_gas=1e22, T_gas=300.0, m_gas=M_AR, eps_max_ev=100.0, seed=seed + 1,
               electron_sid=0, ion_sid=1)
    d = og.Grid.collide(g, [el, ions], mcc, step=9)
    assert d["rc"] == 0
    return el, ions, d, n, e0


def test_ionisation_energy_share_is_uniform(og):
    # Ionisation (Sec. 2.1 MCC; the share law is a stated reading): the
    # energy left after the 15.76 eV threshold is split between the two
    # electrons by one uniform draw, each leaving isotropically.
    el, ions, d, n, e0 = _ionising_run(og)
    k = d["n_ionized"]
    assert k > 5000 and el.n == n + k and ions.n == k
    parent = np.rint(el.xi[n:el.n] / (8.0 / n)).astype(np.int64)
    assert np.array_equal(el.xi[parent], el.xi[n:el.n])
    e_par = 0.5 * ME * _speed2(el, 0, el.n)[parent] / QE
    e_new = 0.5 * ME * _speed2(el, n, el.n) / QE
    avail = e0 - 15.76
    np.testing.assert_allclose(e_par + e_new, avail, rtol=1e-12)
    share = e_par / avail
    assert stats.kstest(share, "uniform").pvalue > 1e-3
    # the two directions: each isotropic, and uncorrelated with each other
    vp = np.stack([el.vr[parent], el.vt[parent], el.vz[parent]])
    vn = np.stack([el.vr[n:el.n], el.vt[n:el.n], el.vz[n:el.n]])
    up = vp / np.linalg.norm(vp, axis=0)
    un = vn / np.linalg.norm(vn, axis=0)
    tol = 5 / math.sqrt(k)
    assert np.abs(up.mean(axis=1)).max() < tol * math.sqrt(1 / 3) * 1.01
    assert np.abs(un.mean(axis=1)).max() < tol * math.sqrt(1 / 3) * 1.01
    assert abs(np.mean(np.sum(up * un, axis=0))) < tol
    for c in range(3):
        assert np.mean(un[c] ** 2) == pytest.approx(1 / 3, abs=5 * math.sqrt(4 / 45 / k))


def test_newborn_ions_follow_the_gas_maxwellian(og):
    # the ion of an ionisation is the target atom, so it takes a velocity
    # from the T_g Maxwellian: each Cartesian component normal with variance
    # kT/M, <v^2> = 3kT/M
    el, ions, d, n, e0 = _ionising_run(og, seed=31)
    k = ions.n
    sig = math.sqrt(KB * 300.0 / M_AR)
    for comp in (ions.vr[:k], ions.vt[:k], ions.vz[:k]):
        assert stats.kstest(comp / sig, "norm").pvalue > 1e-3
    v2 = _speed2(ions, 0, k)
    # the components are independent: v^2 / (kT/M) is chi-square with 3
    # degrees of freedom (normal marginals alone do not show that)
    assert stats.kstest(v2 / sig ** 2, "chi2", args=(3,)).pvalue > 1e-3
    # var(v^2) = 6 (kT/M)^2 for a 3D Maxwellian
    assert np.mean(v2) == pytest.approx(3 * sig ** 2, abs=5 * math.sqrt(6 / k) * sig ** 2)
    # born at the parent's position, with the child's identifier
    assert np.array_equal(ions.xi[:k], el.xi[n:el.n])
    assert np.array_equal(ions.uid[:k], el.uid[n:el.n])
    assert all(og.child_uid(int(el.uid[p]), 9) == int(u)
               for p, u in zip(np.rint(ions.xi[:50] / (8.0 / n)).astype(np.int64), ions.uid[:50]))
