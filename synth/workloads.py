"""Detector geometries, event recipes and method settings of the synthetic
workloads.  Plain values only: both the GPU library and the CPU oracle
receive them as arguments; nothing here computes any part of the method.

The paper's sample (simulated ttbar events with 70 pile-up collisions in the
CMS-2017 geometry, Section 3) is not available, so seeded synthetic events of
the shapes below stand in for it.
"""
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

KAPPA = 0.299792458e-2  # GeV / (T cm): rho = pT / (KAPPA |q| B)

BARREL, DISK = 0, 1


@dataclass(frozen=True)
class Layer:
    kind: int          # BARREL or DISK
    pos: float         # radius (barrel) or signed z (disk), cm
    ext_lo: float      # barrel: lowest z; disk: inner radius
    ext_hi: float      # barrel: highest z; disk: outer radius
    var_u_max: float   # bound on the hit covariance's u-u term on this layer, cm^2
    var_v_max: float   # bound on its v-v term, cm^2
    n_phi_bins: int = 256
    n_q_bins: int = 16
    # stereo layer: strips measuring along a direction turned by `stereo`
    # (rad) from u towards v, with resolution sigma_perp (cm) across them
    stereo: float = 0.0
    sigma_perp: float = 0.0
    # no sensors for hole_lo < q < hole_hi (q: z on a barrel, r on a disk)
    hole_lo: float = 0.0
    hole_hi: float = 0.0


BARREL_RADII = (4.0, 7.0, 11.0, 16.0, 25.0, 34.0, 43.0, 52.0, 61.0, 70.0)
DISK_Z = tuple(120.0 + 20.0 * i for i in range(9))

SIGMA_RPHI = 0.003   # cm, barrel and disk
SIGMA_Z = 0.01       # cm, barrel
SIGMA_R = 0.01       # cm, disk (the workload leaves it open; same as z)


def barrel_layers(half_len: float = 100.0) -> List[Layer]:
    return [Layer(BARREL, r, -half_len, half_len, SIGMA_RPHI ** 2, SIGMA_Z ** 2)
            for r in BARREL_RADII]


def disk_layers(r_min: float = 20.0, r_max: float = 110.0) -> List[Layer]:
    plus = [Layer(DISK, z, r_min, r_max, SIGMA_RPHI ** 2, SIGMA_R ** 2) for z in DISK_Z]
    minus = [Layer(DISK, -z, r_min, r_max, SIGMA_RPHI ** 2, SIGMA_R ** 2) for z in DISK_Z]
    return plus + minus


@dataclass(frozen=True)
class FindConfig:
    """Settings of the method (all readings of the paper's unstated
    values)."""
    bz: float = 3.8
    kappa: float = KAPPA
    chi2_cut: float = 30.0
    n_cand: int = 6
    max_holes: int = 3
    ms_sigma: float = 0.001
    edge_margin: float = 2.0
    l_min: float = 1e-4
    # diagonal seed prior: x, y, z (cm^2), q/pT ((c/GeV)^2), phi, theta (rad^2).
    # It must be wide against what the three seed hits measure, since it is
    # centred on the triplet estimate itself and would otherwise count the
    # same data twice.
    init_var: Tuple[float, ...] = (1.0, 1.0, 1.0, 1.0, 0.01, 0.01)


@dataclass(frozen=True)
class SeedingConfig:
    """Cuts of the combinatorial triplet seeding (readings; the paper takes
    seeds from outside): three barrel layers, innermost first; pT above
    pt_min (GeV/c); the circle within d0_max (cm) of the beam line; the
    middle hit within dz_max (cm) of the s-z line of the outer two; |z| at
    the point of closest approach below z0_max (cm)."""
    layers: Tuple[int, int, int] = (0, 1, 2)
    pt_min: float = 0.25
    d0_max: float = 0.1
    z0_max: float = 20.0
    dz_max: float = 0.1


@dataclass(frozen=True)
class CleaningConfig:
    """Seed cleaning (readings): seeds sharing a hit are instances of one
    particle if their fitted q/pT agree within tol_ipt (relative), eta
    within tol_eta and phi within tol_phi (rad)."""
    tol_ipt: float = 0.1
    tol_eta: float = 0.02
    tol_phi: float = 0.02


@dataclass(frozen=True)
class EventRecipe:
    pt_lo: float = 0.5
    pt_hi: float = 10.0
    eta_max: float = 0.8
    sigma_vxy: float = 0.01
    sigma_vz: float = 5.0
    ms_sigma: float = 0.0
    hit_ineff: float = 0.0
    noise_frac: float = 0.0


PION_MASS = 0.13957  # GeV


@dataclass(frozen=True)
class MaterialMap:
    """Material in r-z (the paper's 2-D radiation and interaction length
    arrays, Section 2.1): bin (iz, ir) covers r in [ir, ir + 1) r_max / n_r
    and z in -z_max + [iz, iz + 1) 2 z_max / n_z (outside: the nearest edge
    bin) and holds the thickness of the layer crossed there, at normal
    incidence, in radiation lengths (x_x0) and in g/cm^2 (xi)."""
    n_r: int
    n_z: int
    r_max: float
    z_max: float
    x_x0: np.ndarray = field(compare=False)   # [n_z][n_r]
    xi: np.ndarray = field(compare=False)     # [n_z][n_r]
    mass: float = PION_MASS
    k_max: float = 10.0


def material_map(r_max: float, z_max: float, n_r: int, n_z: int, x_x0: float, xi: float,
                 outer_z: float = 50.0, outer_factor: float = 1.5) -> MaterialMap:
    """A map with x_x0 and xi everywhere, times outer_factor where the bin
    lies beyond |z| = outer_z (thicker services at the barrel's ends)."""
    zc = -z_max + (np.arange(n_z) + 0.5) * (2.0 * z_max / n_z)
    f = np.where(np.abs(zc) > outer_z, outer_factor, 1.0)[:, None] * np.ones((1, n_r))
    return MaterialMap(n_r, n_z, r_max, z_max, (x_x0 * f).astype(np.float32),
                       (xi * f).astype(np.float32))


@dataclass(frozen=True)
class FieldMap:
    """Parameterised field: Bz(r, z) = b0 (1 + c_r2 r^2 + c_z2 z^2 +
    c_z4 z^4) tesla (r, z in cm), the radial component neglected; the
    transport takes Runge-Kutta steps of at most h_max cm of transverse
    path."""
    b0: float
    c_r2: float = 0.0
    c_z2: float = 0.0
    c_z4: float = 0.0
    h_max: float = 5.0


@dataclass(frozen=True)
class Workload:
    name: str
    layers: Tuple[Layer, ...]
    recipe: EventRecipe
    find: FindConfig
    n_events: int
    n_tracks: Tuple[int, int]   # (lo, hi); lo == hi means fixed, else log-uniform
    master_seed: int
    # material map (replaces the recipe's and the settings' constant
    # scattering angle), or None
    material: Optional[MaterialMap] = None
    # parameterised field (replaces the settings' uniform bz), or None
    field: Optional[FieldMap] = None


def stereo_layer(layer: Layer, angle: float, sigma_perp: float) -> Layer:
    """The layer with strips turned by `angle`: a hit measures along them
    with SIGMA_RPHI and across them with sigma_perp; the covariance bounds
    are those of the turned covariance."""
    c, s = np.cos(angle), np.sin(angle)
    vw, vp = SIGMA_RPHI ** 2, sigma_perp ** 2
    return replace(layer, stereo=angle, sigma_perp=sigma_perp,
                   var_u_max=c * c * vw + s * s * vp, var_v_max=s * s * vw + c * c * vp)


@dataclass(frozen=True)
class Region:
    """A tracking region's steering: seeds with eta_lo <= eta < eta_hi
    follow `layers` (layer ids) in this order."""
    eta_lo: float
    eta_hi: float
    layers: Tuple[int, ...]


def five_regions(eta_barrel: float = 0.9, eta_endcap: float = 1.7,
                 n_barrel: int = len(BARREL_RADII), n_disks: int = len(DISK_Z),
                 endcap_barrel: int = 7) -> Tuple[Region, ...]:
    """Five eta regions (barrel, -z/+z transition, -z/+z endcap) on the
    layer order of barrel_layers() + disk_layers(): barrel layers by radius,
    then the side's disks by |z|.  The disks start beyond the barrel's end,
    so an outgoing track meets the layers in this order.  The endcap lists
    hold the first `endcap_barrel` barrel layers only."""
    barrel = tuple(range(n_barrel))
    plus = tuple(range(n_barrel, n_barrel + n_disks))
    minus = tuple(range(n_barrel + n_disks, n_barrel + 2 * n_disks))
    inner = barrel[:endcap_barrel]
    big = float(np.finfo(np.float32).max)
    return (Region(-big, -eta_endcap, inner + minus),
            Region(-eta_endcap, -eta_barrel, barrel + minus),
            Region(-eta_barrel, eta_barrel, barrel),
            Region(eta_barrel, eta_endcap, barrel + plus),
            Region(eta_endcap, big, inner + plus))


def cms_like(n_events: int = 10, n_tracks: int = 2000) -> Workload:
    """The realistic recipe on a geometry with the generality of the
    paper's layer description (Section 2.1): barrel layers 4 and 6 (R = 25,
    43 cm) are stereo layers (strips turned by 0.1 rad, 1.5 cm across),
    barrel layer 5 (R = 34 cm) has no sensors for |z| < 2 cm, and every
    disk has a ring without sensors at 50 < r < 55 cm."""
    bl = barrel_layers()
    bl[4] = stereo_layer(bl[4], 0.1, 1.5)
    bl[6] = stereo_layer(bl[6], 0.1, 1.5)
    bl[5] = replace(bl[5], hole_lo=-2.0, hole_hi=2.0)
    dl = [replace(d, hole_lo=50.0, hole_hi=55.0) for d in disk_layers()]
    return Workload(
        name=f"cms_like_{n_events}x{n_tracks}",
        layers=tuple(bl + dl),
        recipe=EventRecipe(pt_lo=0.3, pt_hi=10.0, eta_max=2.4, ms_sigma=0.001,
                           hit_ineff=0.02, noise_frac=0.3),
        find=FindConfig(),
        n_events=n_events, n_tracks=(n_tracks, n_tracks), master_seed=0x5EED0007)


def barrel_material(n_tracks: int = 300) -> Workload:
    """The small barrel's 10 cylinders with heavy material (3% of a
    radiation length and 0.5 g/cm^2 per layer at normal incidence, 1.5x
    beyond |z| = 50 cm), pT 0.5-2 GeV/c: ionisation loss of the order of
    the momentum resolution.  No noise, no inefficiency."""
    return Workload(
        name=f"barrel10_material_1x{n_tracks}",
        layers=tuple(barrel_layers()),
        recipe=EventRecipe(pt_lo=0.5, pt_hi=2.0),
        find=FindConfig(),
        n_events=1, n_tracks=(n_tracks, n_tracks), master_seed=0x5EED0009,
        material=material_map(80.0, 100.0, 16, 8, 0.03, 0.5))


def cms_like_material(n_events: int = 10, n_tracks: int = 2000) -> Workload:
    """The CMS-like geometry with a silicon-like material map (1.5% of a
    radiation length and 0.1 g/cm^2 per layer, 1.5x beyond |z| = 50 cm) in
    place of the constant scattering angle."""
    w = cms_like(n_events, n_tracks)
    return replace(w, name=f"cms_like_material_{n_events}x{n_tracks}",
                   material=material_map(120.0, 300.0, 24, 30, 0.015, 0.1))


def solenoid_field() -> FieldMap:
    """A solenoid-like axial field: 3.8 T at the centre, 5% lower at the
    barrel's ends (|z| = 100 cm), 45% lower at the last disks (|z| = 280
    cm), 1% lower at r = 100 cm."""
    return FieldMap(b0=3.8, c_r2=-1e-6, c_z2=-4.9e-6, c_z4=-1.1e-11)


def barrel_endcap_field(n_events: int = 10, n_tracks: int = 2000) -> Workload:
    """The realistic barrel + endcap recipe in the solenoid-like field."""
    w = barrel_endcap(n_events, n_tracks)
    return replace(w, name=f"barrel10_disk18_field_{n_events}x{n_tracks}",
                   master_seed=0x5EED000B, field=solenoid_field())


def small_barrel() -> Workload:
    """1 event, 200 tracks, 10 cylinders, no material, no noise."""
    return Workload(
        name="barrel10_1x200",
        layers=tuple(barrel_layers()),
        recipe=EventRecipe(),
        find=FindConfig(ms_sigma=0.0),
        n_events=1, n_tracks=(200, 200), master_seed=0x5EED0001)


def barrel_endcap(n_events: int = 100, n_tracks: int = 5000) -> Workload:
    """Barrel + 2x9 disks; 100 events x 5,000 tracks; scattering,
    inefficiency and noise."""
    return Workload(
        name=f"barrel10_disk18_{n_events}x{n_tracks}",
        layers=tuple(barrel_layers() + disk_layers()),
        recipe=EventRecipe(pt_lo=0.3, pt_hi=10.0, eta_max=2.4, ms_sigma=0.001,
                           hit_ineff=0.02, noise_frac=0.3),
        find=FindConfig(),
        n_events=n_events, n_tracks=(n_tracks, n_tracks), master_seed=0x5EED0002)


def batched_uneven(n_events: int = 512) -> Workload:
    """Many events of uneven size: track counts log-uniform in 500-20,000."""
    w = barrel_endcap()
    return replace(w, name=f"barrel10_disk18_{n_events}x500-20000",
                   n_events=n_events, n_tracks=(500, 20000), master_seed=0x5EED0003)


def dense(n_events: int = 4) -> Workload:
    """Dense finding events: 25,000 tracks with 50% noise."""
    w = barrel_endcap()
    return replace(w, name=f"barrel10_disk18_{n_events}x25000_noise50",
                   recipe=replace(w.recipe, noise_frac=0.5),
                   n_events=n_events, n_tracks=(25000, 25000), master_seed=0x5EED0005)


def layer_arrays(layers) -> dict:
    """Columns of a layer list, for marshalling."""
    return {
        "kind": np.array([l.kind for l in layers], np.int32),
        "pos": np.array([l.pos for l in layers], np.float64),
        "ext_lo": np.array([l.ext_lo for l in layers], np.float64),
        "ext_hi": np.array([l.ext_hi for l in layers], np.float64),
        "var_u_max": np.array([l.var_u_max for l in layers], np.float64),
        "var_v_max": np.array([l.var_v_max for l in layers], np.float64),
        "n_phi_bins": np.array([l.n_phi_bins for l in layers], np.int32),
        "n_q_bins": np.array([l.n_q_bins for l in layers], np.int32),
    }
