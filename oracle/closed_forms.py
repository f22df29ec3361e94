"""Closed-form surface pressures and identities that pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle.py``).

Conventions: outward normal, time factor e^{-i w t}, outgoing waves
h_n^{(1)}, g = dp/dn on the surface.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sps


def sph_h1(n, z):
    return sps.spherical_jn(n, z) + 1j * sps.spherical_yn(n, z)


def sph_h1p(n, z):
    return sps.spherical_jn(n, z, derivative=True) + 1j * sps.spherical_yn(n, z, derivative=True)


def sphere_mode_pressure(n, k, a):
    """Surface pressure of the radiating field with dp/dr = Y_n on r = a:
    p(a) = h_n(ka) / (k h_n'(ka)) times the same angular factor."""
    z = k * a
    return sph_h1(n, z) / (k * sph_h1p(n, z))


def pulsating_sphere(k, a, g=1.0):
    """dp/dr = g on r = a:  p(a) = g a / (i k a - 1)."""
    return g * a / (1j * k * a - 1.0)


def pulsating_sphere_field(k, a, r, g=1.0):
    """Exterior field of the pulsating sphere (dp/dr = g on r = a): the
    monopole p(r) = g a^2 e^{ik(r-a)} / ((ika - 1) r), equal to
    pulsating_sphere(k, a, g) at r = a."""
    r = np.asarray(r, dtype=np.float64)
    return g * a * a * np.exp(1j * k * (r - a)) / ((1j * k * a - 1.0) * r)


def oscillating_sphere_factor(k, a):
    """dp/dr = cos(theta) on r = a:  p(a, theta) = F cos(theta) with
    F = a (z + i) / (i z^2 - 2 z - 2 i),  z = k a."""
    z = k * a
    return a * (z + 1j) / (1j * z * z - 2.0 * z - 2.0j)


def point_source_field(k, x, x0):
    """G(x, x0) = e^{ik|x-x0|}/(4 pi |x-x0|) at points x (n,3)."""
    r = np.linalg.norm(np.asarray(x) - np.asarray(x0)[None, :], axis=1)
    return np.exp(1j * k * r) / (4.0 * np.pi * r)


def point_source_normal_derivative(k, x, n, x0):
    """d/dn_x G(x, x0) at points x with normals n."""
    x = np.asarray(x)
    d = x - np.asarray(x0)[None, :]
    r = np.linalg.norm(d, axis=1)
    g1 = np.exp(1j * k * r) * (1j * k * r - 1.0) / (4.0 * np.pi * r * r)
    return g1 * np.einsum("ij,ij->i", d, np.asarray(n)) / r


def sphere_single_layer_of_one(k, a):
    """int_{|y|=a} G(x,y) dS(y) for |x| = a: e^{ika} sin(ka)/k  (a at k = 0)."""
    if k == 0.0:
        return a
    return np.exp(1j * k * a) * np.sin(k * a) / k


def flat_disk_G_integral(k, eps):
    """int over a flat disk of radius eps of e^{ikr}/(4 pi r) about its centre."""
    if k == 0.0:
        return eps / 2.0
    return (np.exp(1j * k * eps) - 1.0) / (2j * k)
