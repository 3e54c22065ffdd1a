"""Seeded synthetic workloads for the RF-ablation bioheat stepper.

This module only *generates inputs*: voxel label volumes, per-label tissue
parameters, needle polylines with per-tine powers, time step and step count.
It contains none of the method's arithmetic (no source rasterisation, no
stencil, no damage model), so both the FP64 oracle and the HIP library can be
driven from the same inputs without sharing any computation.

Workloads stand in for the paper's data, which is not available: the
segmented liver CT volume (Sec. "Implementation": 256^2 x 234 voxels) is
replaced by a liver background with a spherical tumour and random
cylindrical vessels, and the paper's Dirichlet needle tip (Sec. "Evaluation
Methods") by Gaussian line sources of given power, one per tine.

Layout everywhere: C order [x][y][z], z fastest.  Positions are metres in a
frame whose origin is the grid centre; voxel i along an axis of n voxels and
spacing d sits at (2 i - (n - 1)) d / 2, so mirrored voxels have exactly
negated coordinates.

Label convention used by every case here:
    0 boundary  outer voxel layer, held at 37 degC, not tissue
    1 liver     background parenchyma
    2 tumour    spherical lesion
    3 vessel    cylindrical heat sink (high perfusion)
Label priority: boundary > vessel > tumour > liver.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Blood properties used to turn a perfusion rate w_b [1/s] into the
# volumetric perfusion coefficient h = rho_b c_b w_b [W/m^3/K].  The paper
# gives c_b = 3617 J/kg/K (Sec. "Specialized Methods") but no blood density;
# rho_b = 1050 kg/m^3 is the assumed value.
RHO_BLOOD = 1050.0
C_BLOOD = 3617.0

# Liver thermal properties of the workloads (k, rho, c) in SI units.
K_LIVER, RHO_LIVER, C_LIVER = 0.52, 1060.0, 3600.0
K_TUMOUR = 0.57
W_LIVER, W_TUMOUR, W_VESSEL = 0.0064, 0.002, 0.05  # perfusion rates, 1/s

# Damage model parameters (Arrhenius frequency factor and activation energy),
# gas constant and the instantaneous-necrosis threshold.
ARRHENIUS_A = 7.39e39
ARRHENIUS_EA = 2.577e5
GAS_R = 8.314
T_DEATH = 60.0
OMEGA_CAP = 1e30
T_BLOOD = 37.0

LABEL_BOUNDARY, LABEL_LIVER, LABEL_TUMOUR, LABEL_VESSEL = 0, 1, 2, 3


@dataclasses.dataclass
class Tissue:
    """Per-label parameters: k [W/m/K], rho [kg/m^3], c [J/kg/K],
    h [W/m^3/K] (= rho_b c_b w_b), q_met [W/m^3], t_fixed [degC] (used when
    fixed), fixed (voxel keeps its value), tissue (voxel accumulates damage)."""
    k: float
    rho: float
    c: float
    h: float
    q_met: float = 0.0
    t_fixed: float = 37.0
    fixed: int = 0
    tissue: int = 1


@dataclasses.dataclass
class Needle:
    """Needle as tines; tine t is the polyline pts[pt_offset[t]:pt_offset[t+1]]
    (metres, grid-centre frame) carrying power[t] watts, smeared by an
    isotropic Gaussian of standard deviation sigma [m]."""
    pt_offset: np.ndarray  # int32 [n_tines + 1]
    pts: np.ndarray        # float64 [n_points, 3]
    power: np.ndarray      # float64 [n_tines]
    sigma: float
    kind: str = "straight"

    @property
    def n_tines(self) -> int:
        return int(len(self.power))


@dataclasses.dataclass
class Case:
    name: str
    shape: tuple            # (nx, ny, nz)
    spacing: tuple          # (dx, dy, dz) metres
    labels: np.ndarray      # uint8 [nx, ny, nz]
    tissue: List[Tissue]
    needle: Needle
    dt: float
    n_steps: int
    seed: int
    t_death: float = T_DEATH
    arrhenius_a: float = ARRHENIUS_A
    arrhenius_ea: float = ARRHENIUS_EA
    gas_r: float = GAS_R
    omega_cap: float = OMEGA_CAP
    t_blood: float = T_BLOOD
    # perfusion scaled by the surviving cell fraction exp(-Omega) (Linte's
    # tissue-state factor; off in the planning workloads, as in the paper's
    # own model)
    perfusion_decay: bool = False
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_voxels(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


def perfusion_coefficient(w_b: float) -> float:
    """Volumetric perfusion coefficient rho_b c_b w_b for a rate w_b [1/s]."""
    return RHO_BLOOD * C_BLOOD * w_b


def standard_tissue() -> List[Tissue]:
    """Label table shared by all cases (boundary, liver, tumour, vessel)."""
    return [
        Tissue(K_LIVER, RHO_LIVER, C_LIVER, 0.0, 0.0, 37.0, fixed=1, tissue=0),
        Tissue(K_LIVER, RHO_LIVER, C_LIVER, perfusion_coefficient(W_LIVER)),
        Tissue(K_TUMOUR, RHO_LIVER, C_LIVER, perfusion_coefficient(W_TUMOUR)),
        Tissue(K_LIVER, RHO_LIVER, C_LIVER, perfusion_coefficient(W_VESSEL)),
    ]


def voxel_axes(shape: Sequence[int], spacing: Sequence[float]):
    """Voxel-centre coordinates per axis, (2 i - (n - 1)) d / 2."""
    return [(2.0 * np.arange(n) - (n - 1)) * d / 2.0 for n, d in zip(shape, spacing)]


def _with_boundary(labels: np.ndarray) -> np.ndarray:
    labels[0, :, :] = labels[-1, :, :] = LABEL_BOUNDARY
    labels[:, 0, :] = labels[:, -1, :] = LABEL_BOUNDARY
    labels[:, :, 0] = labels[:, :, -1] = LABEL_BOUNDARY
    return labels


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def _random_cap_direction(rng: np.random.Generator, max_deg: float) -> np.ndarray:
    """Direction uniform on the spherical cap of half-angle max_deg around +z."""
    cmin = math.cos(math.radians(max_deg))
    cz = rng.uniform(cmin, 1.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    s = math.sqrt(max(0.0, 1.0 - cz * cz))
    return np.array([s * math.cos(phi), s * math.sin(phi), cz])


def _random_unit(rng: np.random.Generator) -> np.ndarray:
    cz = rng.uniform(-1.0, 1.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    s = math.sqrt(max(0.0, 1.0 - cz * cz))
    return np.array([s * math.cos(phi), s * math.sin(phi), cz])


def _random_in_ball(rng: np.random.Generator, radius: float) -> np.ndarray:
    return _random_unit(rng) * radius * rng.uniform(0.0, 1.0) ** (1.0 / 3.0)


def straight_needle(tip, direction, active_len: float, power: float,
                    sigma: float) -> Needle:
    """One tine: the active electrode is the segment [tip - L u, tip]."""
    u = _unit(direction)
    tip = np.asarray(tip, dtype=np.float64)
    pts = np.stack([tip - active_len * u, tip])
    return Needle(np.array([0, 2], dtype=np.int32), pts,
                  np.array([power], dtype=np.float64), sigma, "straight")


def umbrella_needle(rng: np.random.Generator, tip, direction, n_tines: int,
                    total_power: float, sigma: float, r_min=8e-3, r_max=15e-3,
                    jitter_deg=5.0, n_chords=64, sweep=2.0 * math.pi / 3.0) -> Needle:
    """Tines leave the tip at azimuth 2 pi k / n (+ uniform jitter) as
    circular arcs of radius R_k ~ U(r_min, r_max), tangent to the shaft at
    the tip, curving outward and back over `sweep` radians; each arc is a
    polyline of n_chords chords.  Power is shared in proportion to length."""
    u = _unit(direction)
    tip = np.asarray(tip, dtype=np.float64)
    helper = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    v = _unit(np.cross(u, helper))
    w = np.cross(u, v)
    pts, offs, lens = [], [0], []
    for k in range(n_tines):
        phi = 2.0 * math.pi * k / n_tines + math.radians(rng.uniform(-jitter_deg, jitter_deg))
        e = math.cos(phi) * v + math.sin(phi) * w
        radius = rng.uniform(r_min, r_max)
        t = np.linspace(0.0, sweep, n_chords + 1)
        arc = tip[None, :] + radius * (1.0 - np.cos(t))[:, None] * e[None, :] \
            + radius * np.sin(t)[:, None] * u[None, :]
        pts.append(arc)
        offs.append(offs[-1] + n_chords + 1)
        lens.append(radius * sweep)
    lens = np.asarray(lens)
    power = total_power * lens / lens.sum()
    return Needle(np.asarray(offs, dtype=np.int32), np.concatenate(pts), power,
                  sigma, f"umbrella{n_tines}")


def tissue_labels(rng: np.random.Generator, shape, spacing, tumour_centre,
                  tumour_radius, n_vessels, r_vessel=(1e-3, 3e-3)):
    """Liver background, one spherical tumour, random infinite cylindrical
    vessels through uniform points of the box with uniform directions."""
    ax = voxel_axes(shape, spacing)
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    labels = np.full(shape, LABEL_LIVER, dtype=np.uint8)
    c = np.asarray(tumour_centre)
    r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
    labels[r2 <= tumour_radius ** 2] = LABEL_TUMOUR
    half = np.array([a[-1] for a in ax])
    vessels = []
    for _ in range(n_vessels):
        p = rng.uniform(-half, half)
        d = _random_unit(rng)
        rv = rng.uniform(*r_vessel)
        rx, ry, rz = X - p[0], Y - p[1], Z - p[2]
        along = rx * d[0] + ry * d[1] + rz * d[2]
        perp2 = rx * rx + ry * ry + rz * rz - along * along
        labels[perp2 <= rv * rv] = LABEL_VESSEL
        vessels.append((p.tolist(), d.tolist(), rv))
    return _with_boundary(labels), vessels


# ----------------------------------------------------------------------------
# The five workloads.  Seeds are 1000 * config + instance.
# ----------------------------------------------------------------------------

def case_homogeneous(n: int = 32, dx: float = 1e-3, power: float = 20.0,
                     sigma: float = 1e-3, active_len: float = 10e-3,
                     dt: float = 0.05, n_steps: int = 1000, seed: int = 1000) -> Case:
    """Homogeneous liver cube with a Dirichlet 37 degC outer layer and one
    straight needle along +z through the centre, active segment centred on
    the grid centre (so the case is mirror symmetric in x, y, z and x<->y).
    Defaults: 32^3 at 1 mm, 20 W, sigma 1 mm, 10 mm tip, 1000 x 0.05 s."""
    shape = (n, n, n)
    labels = _with_boundary(np.full(shape, LABEL_LIVER, dtype=np.uint8))
    needle = straight_needle([0.0, 0.0, active_len / 2.0], [0.0, 0.0, 1.0],
                             active_len, power, sigma)
    return Case("homogeneous", shape, (dx, dx, dx), labels, standard_tissue()[:2],
                needle, dt, n_steps, seed)


# The paper's own liver model and evaluation setting (Sec. "Specialized
# Methods for Liver Ablation Simulation": the constants listed after Eq.
# (2675-eq1_Kath); Sec. "Evaluation Methods": 0.5 mm voxels, dt 0.1 s, a
# hemispherical electrode tip held at 90 or 60 degC).  The planning
# workloads above use the configured values instead.
PAPER_K, PAPER_RHO, PAPER_C = 0.52, 1079.0, 3540.0
PAPER_WB, PAPER_CB = 16.687, 3617.0     # w_b [kg/m^3/s] and c_b [J/kg/K]
PAPER_QM = 10714.0                       # metabolic heat, W/m^3
PAPER_R = 8.31                           # gas constant as printed
LABEL_TIP = 2                            # class of the held electrode tip (paper mode)


def paper_tip_offsets() -> np.ndarray:
    """Voxel offsets (i, j, k) of the hemispherical electrode tip, 5 x 5 x 3
    voxels: (i / 2.5)^2 + (j / 2.5)^2 + (k / 3)^2 <= 1 with k = 0, 1, 2 (the
    flat face at k = 0, the dome toward +z)."""
    r = range(-2, 3)
    return np.array([(i, j, k) for i in r for j in r for k in range(3)
                     if (i / 2.5) ** 2 + (j / 2.5) ** 2 + (k / 3.0) ** 2 <= 1.0], dtype=np.int64)


def case_paper_mode(tip_c: float = 90.0, n: int = 48, dx: float = 0.5e-3, dt: float = 0.1,
                    n_steps: int = 600, seed: int = 6000) -> Case:
    """The paper's evaluation setting: homogeneous liver with the paper's
    constants (perfusion h = w_b c_b, metabolic heat Q_m, R as printed), a
    hemispherical tip of 5 x 5 x 3 voxels held at tip_c degC at the grid
    centre (class LABEL_TIP: held, no damage), no RF source, everything else
    starting at 37 degC with a held 37 degC outer layer.  Probe points:
    paper_probes()."""
    shape = (n, n, n)
    labels = _with_boundary(np.full(shape, LABEL_LIVER, dtype=np.uint8))
    c = n // 2
    for i, j, k in paper_tip_offsets():
        labels[c + i, c + j, c + k] = LABEL_TIP
    h = PAPER_WB * PAPER_CB
    tissue = [Tissue(PAPER_K, PAPER_RHO, PAPER_C, 0.0, 0.0, 37.0, fixed=1, tissue=0),
              Tissue(PAPER_K, PAPER_RHO, PAPER_C, h, PAPER_QM),
              Tissue(PAPER_K, PAPER_RHO, PAPER_C, 0.0, 0.0, float(tip_c), fixed=1, tissue=0)]
    none = Needle(np.array([0], np.int32), np.zeros((0, 3)), np.zeros(0), dx, "none")
    return Case(f"paper_tip{tip_c:g}", shape, (dx, dx, dx), labels, tissue, none, dt, n_steps,
                seed, gas_r=PAPER_R, meta={"tip_c": float(tip_c)})


def paper_probes(case: Case, distances_mm=(2.5, 5.0)) -> dict:
    """Voxel index of each probe: on the tip axis, the given distance beyond
    the dome's apex voxel (distances in whole voxels of the case's spacing)."""
    n = case.shape[0]
    c = n // 2
    apex = c + int(paper_tip_offsets()[:, 2].max())
    dz = case.spacing[2] * 1e3
    return {d: (c, c, apex + int(round(d / dz))) for d in distances_mm}


def breathing_field(shape, spacing, amplitude_m: float = 5e-3, seed: int = 7000) -> np.ndarray:
    """Synthetic inverse breathing displacement v [3, nx, ny, nz] (float32,
    metres), a stand-in for the 4D-CT registration fields the paper uses:
    mostly cranio-caudal (z), largest mid-grid, zero normal motion at the
    walls, smooth enough to stay diffeomorphic (|dv/dx| below 0.5 at 5 mm over
    a few centimetres).  A seeded random phase varies the pattern."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=3)
    u = [np.linspace(0.0, 1.0, n) for n in shape]
    X, Y, Z = np.meshgrid(*u, indexing="ij")
    bump = np.sin(np.pi * X) * np.sin(np.pi * Y)
    vz = amplitude_m * bump * np.sin(np.pi * Z)
    vx = 0.3 * amplitude_m * np.sin(np.pi * X) * np.sin(2 * np.pi * Y + ph[0]) * np.sin(np.pi * Z)
    vy = 0.2 * amplitude_m * np.sin(2 * np.pi * X + ph[1]) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
    return np.stack([vx, vy, vz]).astype(np.float32)


def breathing_surrogate(t: float, period_s: float = 4.0) -> float:
    """Surrogate signal of a regular breathing cycle in [0, 1]."""
    return float(np.sin(np.pi * t / period_s) ** 2)


def hot_field(shape, spacing, peak_c: float = 900.0, sigma_m: float = 4e-3,
              seed: int = 7100) -> np.ndarray:
    """Synthetic temperature image (degC, float64): 37 degC plus a few
    Gaussian hot spots up to peak_c, steep enough (hundreds of K per voxel
    near the peaks) to exercise an interpolation."""
    rng = np.random.default_rng(seed)
    axes = voxel_axes(shape, spacing)
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    T = np.full(shape, 37.0)
    half = np.array([(n - 1) * d / 2.0 for n, d in zip(shape, spacing)])
    for k in range(3):
        c = rng.uniform(-0.5 * half, 0.5 * half)
        a = peak_c - 37.0 if k == 0 else rng.uniform(50.0, 300.0)
        s = sigma_m * rng.uniform(0.5, 1.5)
        T += a * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * s * s))
    return T


def case_straight(n: int = 128, dx: float = 0.5e-3, dt: float = 0.01,
                  n_steps: int = 1000, seed: int = 2000) -> Case:
    """Heterogeneous liver (tumour r ~ U(6,10) mm centred <= 5 mm from the tip,
    3-6 vessels of radius 1-3 mm), straight needle tipped at the grid centre,
    direction within 30 degrees of +z, P ~ U(15, 40) W, 10 mm active,
    sigma 1 mm.  Defaults: 128^3 at 0.5 mm, 1000 x 0.01 s (10 s)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    tip = np.zeros(3)
    tumour_r = rng.uniform(6e-3, 10e-3)
    tumour_c = tip + _random_in_ball(rng, 5e-3)
    labels, vessels = tissue_labels(rng, shape, (dx,) * 3, tumour_c, tumour_r,
                                    int(rng.integers(3, 7)))
    direction = _random_cap_direction(rng, 30.0)
    power = rng.uniform(15.0, 40.0)
    needle = straight_needle(tip, direction, 10e-3, power, 1e-3)
    return Case("straight", shape, (dx,) * 3, labels, standard_tissue(), needle,
                dt, n_steps, seed,
                meta=dict(tumour_centre=tumour_c.tolist(), tumour_radius=tumour_r,
                          vessels=vessels, direction=direction.tolist()))


def case_umbrella(n: int = 256, dx: float = 0.5e-3, dt: float = 0.01,
                  n_steps: int = 6000, n_tines: int = 9, total_power: float = 60.0,
                  sigma: float = 0.7e-3, seed: int = 3000) -> Case:
    """Same tissue model with a 9-tine umbrella needle (arc radius 8-15 mm,
    +-5 degree azimuth jitter, sigma 0.7 mm, 60 W shared by length).
    Defaults: 256^3 at 0.5 mm, 6000 x 0.01 s (60 s)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    tip = np.zeros(3)
    tumour_r = rng.uniform(6e-3, 10e-3)
    tumour_c = tip + _random_in_ball(rng, 5e-3)
    labels, vessels = tissue_labels(rng, shape, (dx,) * 3, tumour_c, tumour_r,
                                    int(rng.integers(3, 7)))
    direction = _random_cap_direction(rng, 30.0)
    needle = umbrella_needle(rng, tip, direction, n_tines, total_power, sigma)
    return Case("umbrella", shape, (dx,) * 3, labels, standard_tissue(), needle,
                dt, n_steps, seed,
                meta=dict(tumour_centre=tumour_c.tolist(), tumour_radius=tumour_r,
                          vessels=vessels, direction=direction.tolist()))


def case_umbrella_window(n: int = 160, **kw) -> Case:
    """The centred n^3 window of the umbrella workload: the same needle,
    time step and step count and the same tissue labels on the window's
    voxels (voxel centres coincide with the full grid's, since both grids
    are centred), with the window's outer layer held at 37 degC."""
    full = case_umbrella(**kw)
    o = (full.shape[0] - n) // 2
    if o < 0 or (full.shape[0] - n) % 2:
        raise ValueError("the window must be centred inside the full grid")
    labels = _with_boundary(np.ascontiguousarray(full.labels[o:o + n, o:o + n, o:o + n]))
    return dataclasses.replace(full, name=f"umbrella_window{n}", shape=(n, n, n),
                               labels=labels)


def case_planning_instance(instance: int, n_min: int = 64, n_max: int = 160,
                           n_steps: int = 2000, base_seed: int = 4000) -> Case:
    """One instance of the batched planning sweep: cubic grid n ~ U{64..160},
    spacing ~ U(0.5, 1) mm, needle type ~ U{straight, 3-tine, 9-tine},
    tumour centred <= 5 mm from the grid centre, tip uniform in a ball of half
    the tumour radius around the tumour centre, power ~ U(10, 60) W,
    dt = 0.01 s (dx / 0.5 mm)^2."""
    seed = base_seed + instance
    rng = np.random.default_rng(seed)
    n = int(rng.integers(n_min, n_max + 1))
    dx = rng.uniform(0.5e-3, 1e-3)
    shape = (n, n, n)
    tumour_r = rng.uniform(6e-3, 10e-3)
    tumour_c = _random_in_ball(rng, 5e-3)
    tip = tumour_c + _random_in_ball(rng, tumour_r / 2.0)
    labels, vessels = tissue_labels(rng, shape, (dx,) * 3, tumour_c, tumour_r,
                                    int(rng.integers(3, 7)))
    direction = _random_cap_direction(rng, 30.0)
    power = rng.uniform(10.0, 60.0)
    kind = int(rng.integers(0, 3))
    if kind == 0:
        needle = straight_needle(tip, direction, 10e-3, power, 1e-3)
    else:
        needle = umbrella_needle(rng, tip, direction, 3 if kind == 1 else 9, power,
                                 max(0.7e-3, dx))
    dt = 0.01 * (dx / 0.5e-3) ** 2
    return Case(f"planning{instance}", shape, (dx,) * 3, labels, standard_tissue(),
                needle, dt, n_steps, seed,
                meta=dict(tumour_centre=tumour_c.tolist(), tumour_radius=tumour_r,
                          vessels=vessels, kind=needle.kind))


def planning_sweep(n_instances: int = 64, **kw) -> List[Case]:
    return [case_planning_instance(i, **kw) for i in range(n_instances)]


def case_differentiation(n: int = 128, dx: float = 0.5e-3, dt: float = 0.02,
                         n_steps: int = 600, seed: int = 5000,
                         sigma: float = 0.7e-3) -> Case:
    """Differentiation workload: umbrella (9 tines, 60 W shared by length) in
    the seeded tissue model.  A 32^3 copy uses n=32, dx=2 mm and
    sigma = max(sigma, dx).  Defaults: 128^3 at 0.5 mm, 600 x 0.02 s."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    tip = np.zeros(3)
    tumour_r = rng.uniform(6e-3, 10e-3)
    tumour_c = tip + _random_in_ball(rng, 5e-3)
    labels, vessels = tissue_labels(rng, shape, (dx,) * 3, tumour_c, tumour_r,
                                    int(rng.integers(3, 7)))
    direction = _random_cap_direction(rng, 30.0)
    needle = umbrella_needle(rng, tip, direction, 9, 60.0, max(sigma, dx))
    return Case("differentiation", shape, (dx,) * 3, labels, standard_tissue(),
                needle, dt, n_steps, seed,
                meta=dict(tumour_centre=tumour_c.tolist(), tumour_radius=tumour_r,
                          vessels=vessels))


def random_tissue_case(rng_seed: int, shape=(12, 10, 14), spacing=(1e-3, 0.8e-3, 1.2e-3),
                       n_classes: int = 5, n_tines: int = 2, dt: Optional[float] = None,
                       n_steps: int = 20) -> Case:
    """Small fully random case for property tests: random labels (including a
    fixed, non-tissue class held at a random temperature), random parameters,
    anisotropic spacing and a random multi-chord needle."""
    rng = np.random.default_rng(rng_seed)
    tissue = [Tissue(K_LIVER, RHO_LIVER, C_LIVER, 0.0, 0.0, 37.0, fixed=1, tissue=0)]
    for c in range(1, n_classes):
        fixed = int(c == n_classes - 1)
        tissue.append(Tissue(rng.uniform(0.3, 0.8), rng.uniform(900, 1200),
                             rng.uniform(3000, 4000), rng.uniform(0, 2e5),
                             rng.uniform(0, 2e4), rng.uniform(30, 80), fixed=fixed,
                             tissue=int(rng.integers(0, 2)) if fixed else 1))
    labels = rng.integers(1, n_classes, size=shape).astype(np.uint8)
    labels = _with_boundary(labels)
    half = np.array([(n - 1) * d / 2.0 for n, d in zip(shape, spacing)])
    pts, offs = [], [0]
    for _ in range(n_tines):
        m = int(rng.integers(1, 5))
        p = rng.uniform(-half * 0.6, half * 0.6, size=(m + 1, 3))
        pts.append(p)
        offs.append(offs[-1] + m + 1)
    needle = Needle(np.asarray(offs, dtype=np.int32), np.concatenate(pts),
                    rng.uniform(1.0, 10.0, size=n_tines), float(min(spacing)) * 1.2,
                    "random")
    if dt is None:
        dt = 0.01
    return Case(f"random{rng_seed}", tuple(shape), tuple(spacing), labels, tissue,
                needle, dt, n_steps, rng_seed)


def config_case(config: int, **kw) -> Case:
    """Workload by number: 1 homogeneous 32^3, 2 straight 128^3, 3 umbrella
    256^3, 5 differentiation 128^3 (4 is a list: see planning_sweep)."""
    if config == 1:
        return case_homogeneous(**kw)
    if config == 2:
        return case_straight(**kw)
    if config == 3:
        return case_umbrella(**kw)
    if config == 5:
        return case_differentiation(**kw)
    raise ValueError("config 4 is a batch: use planning_sweep()")
