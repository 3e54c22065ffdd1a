"""Closed-form solutions used to pin the FP64 oracle (test helpers only).

None of these share code with the oracle or the HIP library.  Each is an
independent mathematical route to a result the explicit bioheat scheme
(Eq. (CUDAbioheat3d), paper Sec. "Specialized Methods for Liver Ablation
Simulation") must reproduce, exactly or in its continuum limit.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import fft, special


def dst_solution(theta0_int, src_int, K, rho, c, h, spacing, dt, n_steps):
    """Exact n-step solution of the explicit scheme on a homogeneous box
    whose outer voxel layer is held at excess temperature 0.

    The interior (M_d = N_d - 2 voxels per axis) second-difference operator
    is diagonal in the DST-I basis sin(pi m j / (M + 1)) with eigenvalue
    -4 sin^2(pi m / (2 (M + 1))) / dd^2, so one step multiplies mode m by
        lam_m = 1 - dt / (rho c) [K sum_d 4 sin^2(pi m_d / 2(M_d+1)) / dd^2 + h]
    and adds the transformed source increment dt s / (rho c).  After n steps
        theta_hat = lam^n theta0_hat + (1 - lam^n) / (1 - lam) * src_hat.
    theta0_int, src_int: interior arrays [M_x, M_y, M_z]; src in W/m^3.
    Returns the interior excess temperature after n_steps."""
    M = theta0_int.shape
    lam = np.ones(M)
    rc = rho * c
    for ax, (m_ax, d) in enumerate(zip(M, spacing)):
        m = np.arange(1, m_ax + 1)
        s2 = np.sin(np.pi * m / (2.0 * (m_ax + 1))) ** 2
        shape = [1, 1, 1]
        shape[ax] = m_ax
        lam = lam - dt / rc * K * 4.0 * s2.reshape(shape) / d ** 2
    lam = lam - dt / rc * h
    th0 = fft.dstn(theta0_int, type=1, norm="ortho")
    sh = fft.dstn(src_int * dt / rc, type=1, norm="ortho")
    lam_n = lam ** n_steps
    geo = np.where(np.abs(1.0 - lam) > 0, (1.0 - lam_n) / np.where(lam == 1.0, 1.0, 1.0 - lam),
                   float(n_steps))
    out = lam_n * th0 + geo * sh
    return fft.idstn(out, type=1, norm="ortho")


def dst_steady(src_int, K, h, spacing):
    """Steady state of the same discrete operator (n -> infinity)."""
    M = src_int.shape
    denom = np.full(M, float(h))
    for ax, (m_ax, d) in enumerate(zip(M, spacing)):
        m = np.arange(1, m_ax + 1)
        s2 = np.sin(np.pi * m / (2.0 * (m_ax + 1))) ** 2
        shape = [1, 1, 1]
        shape[ax] = m_ax
        denom = denom + K * 4.0 * s2.reshape(shape) / d ** 2
    return fft.idstn(fft.dstn(src_int, type=1, norm="ortho") / denom, type=1, norm="ortho")


def pennes_sphere(r, a, q, K, h):
    """Steady excess temperature of K lap(theta) - h theta + q 1[r<a] = 0 in
    infinite homogeneous tissue (decay rate m = sqrt(h/K)).  Inside:
    q/h + A sinh(mr)/r, outside: B exp(-mr)/r, with A and B fixed by
    continuity of value and radial flux at r = a (solved here as a 2x2
    linear system rather than copied from a table)."""
    m = math.sqrt(h / K)
    # unknowns (A, B):  q/h + A sinh(ma)/a = B e^{-ma}/a
    #                   A d/dr[sinh(mr)/r]_a = B d/dr[e^{-mr}/r]_a
    s, ch, e = math.sinh(m * a), math.cosh(m * a), math.exp(-m * a)
    d_in = (m * ch * a - s) / a ** 2
    d_out = (-m * a - 1.0) * e / a ** 2
    Amat = np.array([[s / a, -e / a], [d_in, -d_out]])
    rhs = np.array([-q / h, 0.0])
    A, B = np.linalg.solve(Amat, rhs)
    r = np.asarray(r, dtype=np.float64)
    inside = q / h + A * np.sinh(m * r) / np.where(r == 0, 1.0, r)
    inside = np.where(r == 0, q / h + A * m, inside)
    outside = B * np.exp(-m * r) / np.where(r == 0, 1.0, r)
    return np.where(r < a, inside, outside)


def gaussian_kernel(r2, amp, sigma0, alpha, t):
    """Free-space heat kernel: an initial Gaussian bump amp exp(-r^2/2 s0^2)
    stays Gaussian, sigma^2 = sigma0^2 + 2 alpha t, amplitude scaled by
    (sigma0/sigma)^3 (Eq. (eq-funda) convolved in 3-D)."""
    s2 = sigma0 ** 2 + 2.0 * alpha * t
    return amp * (sigma0 ** 2 / s2) ** 1.5 * np.exp(-r2 / (2.0 * s2))


def series_slab(z_faces_resistance, t_hot, t_cold):
    """Temperatures at voxel centres of a 1-D chain held at t_hot and t_cold
    at its two end voxels, in steady state: constant flux through resistances
    R_f = dz / K_face in series (Fourier's law for layered media)."""
    R = np.asarray(z_faces_resistance, dtype=np.float64)
    flux = (t_hot - t_cold) / R.sum()
    return t_hot - flux * np.concatenate([[0.0], np.cumsum(R)])


def arrhenius_integral(A, Ea, R, t_c, duration):
    """Damage integral at constant temperature t_c [degC] (Kelvin inside)."""
    return duration * A * math.exp(-Ea / (R * (t_c + 273.15)))
