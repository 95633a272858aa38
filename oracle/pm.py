"""ORACLE — test infrastructure only.

Plain FP64 (numpy) long-range part of the TreePM force, following the
paper's "Particle Mesh" subsection step by step: the particles' mass is
assigned to a periodic mesh, the density is Fourier transformed, multiplied
by the Green's function of the Poisson equation with the Gaussian low-pass
filter exp(-k^2 A_smth^2), and transformed back.  Only the test-suite, the
smoke entry and the benchmark's CPU-baseline leg may use this module; it
shares nothing with the HIP package.

Readings of what the paper leaves open:
  R27 mass assignment: cloud-in-cell (CIC) onto mesh nodes at j*Delta,
      Delta = L/n; forces and potentials are interpolated back with the same
      weights.
  R28 the Green's function is divided by the square of the CIC window
      W(k) = prod_a sinc^2(pi n_a / n) (assignment and interpolation), and
      is zero for k = 0 (mean density removed, periodic Poisson equation).
  R29 the acceleration is -grad(phi) taken in Fourier space, a_k = -i k phi_k,
      with the Nyquist wavenumber's derivative set to zero.
  R30 the potential excludes the particle's own long-range term: its limit
      -G m / (sqrt(pi) r_s) at r -> 0 is subtracted.
"""
import math

import numpy as np


def cic_weights(pos, n, L):
    """Per axis: lower mesh node index and the weight of the upper node
    (R27).  Nodes sit at j*L/n, periodic."""
    u = np.asarray(pos, dtype=np.float64) * (n / L)
    i0 = np.floor(u)
    f = u - i0
    return i0.astype(np.int64) % n, f


def assign(pos, mass, n, L):
    """Mass density on the n^3 mesh (paper: particles assigned to grid
    cells, density binned onto the mesh)."""
    i0, f = cic_weights(pos, n, L)
    rho = np.zeros((n, n, n))
    for dx in (0, 1):
        wx = f[:, 0] if dx else 1.0 - f[:, 0]
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1.0 - f[:, 1]
            for dz in (0, 1):
                wz = f[:, 2] if dz else 1.0 - f[:, 2]
                np.add.at(rho, ((i0[:, 0] + dx) % n, (i0[:, 1] + dy) % n, (i0[:, 2] + dz) % n),
                          mass * wx * wy * wz)
    return rho / (L / n) ** 3


def wavenumbers(n, L):
    """Signed integer wavenumbers of the DFT along one axis and k = 2 pi m / L."""
    m = np.fft.fftfreq(n, d=1.0 / n)
    return m, 2.0 * math.pi * m / L


def green(n, L, G, r_s):
    """phi_k / rho_k = -4 pi G exp(-k^2 r_s^2) / k^2 / W(k)^2 (paper's
    Green's function with the Gaussian filter; R28)."""
    m, k = wavenumbers(n, L)
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    s = np.ones(n)
    nz = m != 0
    s[nz] = np.sin(math.pi * m[nz] / n) / (math.pi * m[nz] / n)
    sx, sy, sz = np.meshgrid(s, s, s, indexing="ij")
    w2 = (sx * sy * sz) ** 4
    g = np.zeros((n, n, n))
    pos = k2 > 0
    g[pos] = -4.0 * math.pi * G * np.exp(-k2[pos] * r_s * r_s) / k2[pos] / w2[pos]
    return g


def mesh_fields(pos, mass, n, L, G, r_s):
    """Long-range potential and acceleration on the mesh nodes: DFT of the
    density, Green's function, -i k for the gradient (R29), inverse DFT."""
    rho_k = np.fft.fftn(assign(pos, mass, n, L))
    phi_k = green(n, L, G, r_s) * rho_k
    m, k = wavenumbers(n, L)
    kd = k.copy()
    kd[m == -n // 2] = 0.0          # Nyquist derivative dropped
    kx, ky, kz = np.meshgrid(kd, kd, kd, indexing="ij")
    phi = np.fft.ifftn(phi_k).real
    acc = [np.fft.ifftn(-1j * kk * phi_k).real for kk in (kx, ky, kz)]
    return phi, acc


def interpolate(field, pos, n, L):
    """CIC interpolation of a mesh field to the positions (R27)."""
    i0, f = cic_weights(pos, n, L)
    out = np.zeros(len(pos))
    for dx in (0, 1):
        wx = f[:, 0] if dx else 1.0 - f[:, 0]
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1.0 - f[:, 1]
            for dz in (0, 1):
                wz = f[:, 2] if dz else 1.0 - f[:, 2]
                out += wx * wy * wz * field[(i0[:, 0] + dx) % n, (i0[:, 1] + dy) % n, (i0[:, 2] + dz) % n]
    return out


def long_range(pos, mass, L, n, G, r_s, targets=None):
    """Long-range acceleration [M,3] and potential [M] at the targets
    (caller-order indices, None = all), paper's "Particle Mesh" subsection."""
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    phi, acc = mesh_fields(pos, mass, n, L, G, r_s)
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    x = pos[idx]
    a = np.stack([interpolate(c, x, n, L) for c in acc], axis=1)
    p = interpolate(phi, x, n, L) + G * mass[idx] / (math.sqrt(math.pi) * r_s)   # R30
    return a, p
