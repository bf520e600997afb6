"""Pins of the oracle's protons and thermal atmosphere (Sect. 2.3 atmospheric
boundary; Sect. 6.1: electrons, positrons and protons with m_p/m_e = 1836,
atmosphere at k_B T / m_e c^2 = 0.3, electrons everywhere and protons below
H at the start):

* the atmosphere's momenta follow the one-dimensional relativistic thermal
  distribution exp(-gamma/Theta): <gamma> = K_0(1/Theta)/K_1(1/Theta) + Theta,
  the virial <u^2/gamma> = Theta, and its distribution function (quadrature);
* a proton and an electron at rest in a uniform frozen field: u = +E t/1836
  and u = -E t (charge and mass);
* the initial state: as many protons as electrons below H, the field the
  linear ramp of a neutral gap;
* Ampere's law from the trajectories of electrons and protons, with the
  charge the atmosphere brings in and the star takes back;
* the atmosphere screens the surface field, which without it grows as the
  imposed current charges the star.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

F = O.FLAGS


@pytest.mark.parametrize("theta,seed", [(0.3, 1), (0.3 / 1836.0, 2), (3.0, 3)])
def test_thermal_momenta_moments(theta, seed):
    from scipy import special
    n = 100_000
    u = np.array([O.atm_momentum(seed, i, 5, theta) for i in range(n)])
    g = np.sqrt(1.0 + u * u)
    b = 1.0 / theta
    mg = special.k0e(b) / special.k1e(b) + theta
    assert abs(g.mean() - mg) < 4.0 * g.std() / math.sqrt(n)
    v = u * u / g
    assert abs(v.mean() - theta) < 4.0 * v.std() / math.sqrt(n)
    assert abs((u > 0).mean() - 0.5) < 4.0 * 0.5 / math.sqrt(n)


def test_thermal_momenta_distribution():
    from scipy import integrate
    theta, n = 0.3, 60_000
    a = np.sort(np.abs([O.atm_momentum(9, i, 0, theta) for i in range(n)]))
    f = lambda x: math.exp(-(math.sqrt(1.0 + x * x) - 1.0) / theta)
    Z = integrate.quad(f, 0, np.inf)[0]
    idx = np.linspace(0, n - 1, 41).astype(int)[1:-1]
    Fx = np.array([integrate.quad(f, 0, q)[0] / Z for q in a[idx]])
    assert np.max(np.abs(Fx - (idx + 0.5) / n)) < 1.63 / math.sqrt(n) * 1.5


def test_proton_and_electron_in_a_uniform_field():
    N, E0, steps = 64, 3.0, 40
    o = O.Oracle(dict(n_cells=N, init_kind=2, flags=F["FIELD_FROZEN"] | F["QED_OFF"], atm_ppc=0))
    lep = dict(cell=np.array([20], np.int32), xi=np.array([0.5]), u=np.zeros(1), w=np.array([-1.0]),
               id=np.array([1], np.uint64))
    o.set_state(lep)
    o.set_protons(dict(cell=np.array([30], np.int32), xi=np.array([0.25]), u=np.zeros(1), w=np.array([1.0]),
                       id=np.array([2], np.uint64)))
    o.set_field(np.full(N, E0), E0)
    o.step(steps)
    ue, up = o.leptons()["u"][0], o.protons()["u"][0]
    assert abs(ue - (-E0 * o.dt * steps)) < 1e-12 * steps
    assert abs(up - E0 * o.dt * steps / 1836.0) < 1e-15 * steps
    assert abs(ue / up + 1836.0) < 1e-9


def test_initial_state_neutral_below_H():
    N, ppc = 512, 4
    o = O.Oracle(dict(n_cells=N, init_kind=4, ppc_init=ppc, ppc_ref=ppc, flags=F["QED_OFF"], seed=7,
                      h_gap_frac=0.8))
    kh = math.ceil(0.8 * N - 1e-9)
    assert o.proton_counts()["n_pro"] == kh * ppc
    assert o.counts()["n_lep"] == N * ppc
    # below H the charge is zero on average: the field is the co-rotation ramp
    # E = h (eta_co = -n_co, s_co = -1 units), up to the macro-particle noise
    E = o.field()
    h = (np.arange(N) + 0.5) * 0.25
    ramp = np.minimum(h, kh * 0.25)
    noise = math.sqrt(2 * ppc * kh) / ppc * 0.25
    assert np.max(np.abs(E[:kh] - ramp[:kh])) < 5 * noise


def _scum(k, x):
    return np.clip(k[None, :] + 1.0 - x[:, None], 0.0, 1.0)


def test_ampere_with_protons_and_atmosphere():
    # E^{n+1} - E^n = -dt (J - j_m), J the current of the continuous
    # trajectories of electrons and protons, with the atmosphere's particles
    # entering at the surface and absorbed ones leaving through it
    N = 256
    o = O.Oracle(dict(n_cells=N, init_kind=4, ppc_init=4, ppc_ref=4, alpha=2.0, flags=F["QED_OFF"], seed=5,
                      atm_ppc=8, atm_temp=0.3))
    o.step(60)
    for _ in range(4):
        A = {**{("l", int(i)): (c + x, w) for i, c, x, w in zip(*(o.leptons()[k] for k in ("id", "cell", "xi", "w")))},
             **{("p", int(i)): (c + x, w) for i, c, x, w in zip(*(o.protons()[k] for k in ("id", "cell", "xi", "w")))}}
        E0 = o.field()
        o.step(1)
        B = {**{("l", int(i)): (c + x, w) for i, c, x, w in zip(*(o.leptons()[k] for k in ("id", "cell", "xi", "w")))},
             **{("p", int(i)): (c + x, w) for i, c, x, w in zip(*(o.protons()[k] for k in ("id", "cell", "xi", "w")))}}
        E1 = o.field()
        x_old, x_new, q = [], [], []
        for key, (xo, w) in A.items():
            xn = B[key][0] if key in B else (-1.0 if xo < N / 2 else N + 1.0)
            x_old.append(xo); x_new.append(xn); q.append(w)
        for key, (xn, w) in B.items():
            if key not in A:
                x_old.append(0.0); x_new.append(xn); q.append(w)
        x_old, x_new, q = map(np.asarray, (x_old, x_new, q))
        k = np.arange(N)
        flux = -(q[:, None] * o.w0 * (_scum(k, x_new) - _scum(k, x_old))).sum(axis=0)
        dE = -(flux - 2.0 * o.s_co * o.dt)
        assert np.max(np.abs((E1 - E0) - dE)) <= len(q) * o.w0 / 2 ** 24


def test_atmosphere_screens_the_surface_field():
    N = 512
    base = dict(n_cells=N, ppc_init=4, ppc_ref=4, alpha=2.0, flags=F["QED_OFF"], seed=3, h_gap_frac=0.8)
    bare = O.Oracle(dict(base, init_kind=0))
    atm = O.Oracle(dict(base, init_kind=4, atm_ppc=8, atm_temp=0.3))
    es = []
    for _ in range(6):
        bare.step(100)
        atm.step(100)
        es.append(atm.Es)
    # without supply the star charges at the imposed current; with the
    # atmosphere the surface field stays bounded
    assert abs(bare.Es) > 100.0
    assert max(abs(v) for v in es) < 0.1 * abs(bare.Es)
    assert abs(es[-1] - es[2]) < 0.02 * abs(bare.Es)
    c = atm.proton_counts()
    assert c["n_atm_e"] > 1000 and c["n_atm_p"] > 10
