"""The brute-force real-space evaluation of Eq. (Enl) with the soft kernel and
the accuracy of the factorisation of Eq. (phi) (both measured, "parity
unpinned": the paper gives no number for either; the values are recorded).

Pins of the brute-force machinery itself: its phi_s table against the kernel
table's own per-ray construction (different meshes and interpolation), and
the tail integrals against the constant-density property (phi integrates to
zero, so the whole integral of phi_s along the diagonal ray is -2 C_s times
the ray's scale, Eq. Depsnl).
"""
import numpy as np
import pytest

import workloads as W
from oracle import bruteforce as B
from oracle import functional as F
from oracle import kernel_table as kt


def test_soft_table_matches_kernel_table_rays(table):
    for qa, qb in [(1.0, 1.0), (0.4, 1.3), (0.2, 2.5)]:
        Q = np.hypot(qa, qb)
        ray = kt.Ray(qa / Q, qb / Q, 1.0, 0.5)
        D = np.array([0.2, 0.7, 0.99, 1.2, 2.0, 4.0, 9.0, 15.0, 40.0])
        got = B.phi_soft(D * qa / Q, D * qb / Q)
        np.testing.assert_allclose(got, ray(D), rtol=2e-6, atol=1e-9)


def test_tail_integral_matches_constant_density_property(table):
    st = B.soft_table()
    # the last angle node is 45 degrees: d1 = d2
    assert abs(B.TH0_DEG + B.DTH_DEG * (B.NTH - 1) - 45.0) < 1e-12
    p2, p4 = st["p2"][-1], st["p4"][-1]
    soft = 4 * np.pi * (0.5 / 3 + p2 / 5 + p4 / 7)          # Int_0^{d_s=1} 4 pi D^2 phi_s dD
    total = soft + st["cum"][-1, 0]
    # phi_aa(k = 0) = -2 C_s / q^3 with Q = sqrt(2) q on the ray: 4 pi Int D^2 phi_s = -2 C_s 2^(3/2)
    expect = -2.0 * table["c_soft"] * 2.0 ** 1.5
    print("  4 pi Int D^2 phi_s dD on the diagonal: %.9f, -2 C_s 2^(3/2) = %.9f" % (total, expect))
    assert abs(total - expect) < 1e-6 * abs(expect)


def test_factorisation_accuracy_recorded(table):
    """P10: |phi_s(q1 r, q2 r) - sum_ab p_a(q1) p_b(q2) phi_s(q_a r, q_b r)| at
    random (q1, q2) on [q_1, q_c], relative to phi_s(0) = phi0 = 0.5."""
    q = table["qmesh"]
    spl = F.CardinalSplines(q)
    rng = np.random.default_rng(11)
    q1 = np.exp(rng.uniform(np.log(q[0]), np.log(q[-1]), 60))
    q2 = np.exp(rng.uniform(np.log(q[0]), np.log(q[-1]), 60))
    p1, _ = spl(q1)
    p2, _ = spl(q2)
    worst = {}
    for r in [0.3, 1.0, 3.0]:
        exact = B.phi_soft(q1 * r, q2 * r)
        grid = B.phi_soft(q[:, None] * r, q[None, :] * r)
        interp = np.einsum("ap,ab,bp->p", p1, grid, p2)
        worst[r] = np.abs(interp - exact).max() / 0.5
        print("  r = %.1f bohr: max |interp - phi_s| / phi0 = %.2e" % (r, worst[r]))
    # recorded: 1.1e-3, 3.5e-4, 3.1e-3; the bound only guards against a broken check
    assert max(worst.values()) < 1e-2


def _smooth_density(N, scale=0.01):
    wl = W.gauss24()
    at = wl.atoms
    a2 = W.Atoms(pos=at.pos, amp=at.amp * scale, width=at.width)
    return W.density_on_grid((N, N, N), wl.cell, a2), wl.cell


def test_bruteforce_real_space_against_factorised(table):
    """P9: the real-space double sum with the soft kernel against the
    factorised FFT evaluation (E_k), on the 12^3 and 24^3 samplings of the
    10 bohr cell with the atom amplitudes scaled by 0.01 (q0 up to about 1.7,
    kernel width above the grid spacing), images to 12 bohr and the continuum
    tail beyond.  The gap must shrink under refinement.  On the undiluted
    12^3 density (q0 up to 5: the kernel is narrower than the 0.83 bohr
    spacing) the grid sum is not an approximation of the integral; its gap is
    only printed."""
    gaps = {}
    for N in (12, 24):
        n, cell = _smooth_density(N)
        bf = B.energy(n, cell, table, rcut=12.0)
        ek, de, _ = F.energy_potential(n, cell, table)
        gaps[N] = (bf["E_bf"] - ek) / abs(ek)
        print("  %d^3 smooth: E_bf %.6e  E_k %.6e  relative gap %.2e  (Delta E %.3e)" % (N, bf["E_bf"], ek, gaps[N], de))
    n, cell = _smooth_density(12, scale=1.0)
    bf = B.energy(n, cell, table, rcut=12.0)
    ek, de, _ = F.energy_potential(n, cell, table)
    print("  12^3 undiluted: E_bf %.6e  E_k %.6e  relative gap %.2e" % (bf["E_bf"], ek, (bf["E_bf"] - ek) / abs(ek)))
    # recorded: -5.2e-4 at 12^3, 2.2e-5 at 24^3 (undiluted 12^3: 6.4)
    assert abs(gaps[24]) < abs(gaps[12])
    assert abs(gaps[24]) < 1e-3
