"""Seeded synthetic protoplanetary-disc inputs for the coagulation update.

This module only makes inputs: per-cell gas state, dust velocities (standing in
for the dust dynamics solver, whose output the collision kernel reads) and an
initial size distribution.  It contains none of the coagulation method's
arithmetic, and it is the only code that the GPU library's tests and the CPU
oracle's tests both use.

Disc shape follows the paper's transition-disc test (Sec. 7, table `params`):
Sigma_g = Sigma_0 R_au^-1 exp[-(5/R_au)^10], Sigma_0 = 250 g cm^-2, M_* = 1 M_sun,
mu = 2.4; vertically isothermal T = 150 K (R/au)^-1/2; Gaussian rho_g(Z) with
H/R = 0.05; MRN initial dust (n(s) ~ s^-3.5) up to 1 micron at dust-to-gas 0.01.
Columns for the vertically integrated kernel follow the paper's single-radius
coagulation test (Sec. 5.1): R = 20 au, T = 36 K, mu = 2.4, alpha = 1e-3,
v_frag = 1 m/s, 200 species.
No public dataset is involved; every random draw is seeded.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# physical constants (CGS)
K_B = 1.380649e-16
M_H = 1.6735575e-24
G_GRAV = 6.67430e-8
M_SUN = 1.98847e33
AU = 1.495978707e13
YEAR = 3.15576e7
SIGMA_H2 = 2.0e-15          # H2 collision cross-section for the molecular mean free path

SEED_ALPHA = 240218471
SEED_FD = 240218472


@dataclass
class DiscConfig:
    name: str
    n_r: int
    n_z: int
    n_bins: int
    s_min: float                 # cm
    s_max: float                 # cm
    alpha: float | tuple = 1e-3  # scalar, or (lo, hi) log-uniform per radial ring
    v_frag: float = 100.0        # cm/s
    steps: int = 1000
    dt: float = 10.0 * YEAR      # s per coagulation call
    rho_m: float = 1.67          # grain material density, g cm^-3
    r_in_au: float = 5.0
    r_out_au: float = 100.0
    z_max_h: float = 3.0
    h_over_r: float = 0.05
    mu: float = 2.4
    sigma0: float = 250.0
    dust_to_gas: float = 0.01
    s_mrn_max: float = 1.0e-4    # cm
    extra: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return self.n_r * self.n_z


CONFIGS = {
    # 64 (R, 5-100 au) x 32 (Z, 0-3H) cells x 100 bins (0.1 um - 10 cm), plain FP64
    "disc64x32_n100": DiscConfig("disc64x32_n100", 64, 32, 100, 1e-5, 10.0, 1e-3, 100.0, 1000),
    # 256 x 128 cells x 150 bins, v_frag = 10 m/s (FP64 vs split-BF16)
    "disc256x128_n150": DiscConfig("disc256x128_n150", 256, 128, 150, 1e-5, 10.0, 1e-3, 1000.0, 1000),
    # adjoint case: the 64 x 32 x 100 disc over 200 steps
    "disc64x32_n100_adj": DiscConfig("disc64x32_n100_adj", 64, 32, 100, 1e-5, 10.0, 1e-3, 100.0, 200),
    # large: 512 x 256 x 200 bins (0.1 um - 1 m), alpha log-uniform per ring
    "disc512x256_n200": DiscConfig("disc512x256_n200", 512, 256, 200, 1e-5, 100.0, (1e-4, 1e-2), 300.0, 500),
}


def scaled(cfg: DiscConfig, n_r: int, n_z: int, n_bins: int | None = None) -> DiscConfig:
    """Same physics on a coarser cell grid (and optionally fewer bins)."""
    d = dict(cfg.__dict__)
    d.update(name=f"{cfg.name}_sub{n_r}x{n_z}", n_r=n_r, n_z=n_z)
    if n_bins is not None:
        d["n_bins"] = n_bins
    return DiscConfig(**d)


def make_cells(cfg: DiscConfig):
    """Per-cell gas state, cell index c = i_r * n_z + i_z (radius-major).

    Returns dict with R, Z (cm), Sigma_g, and the seven per-cell inputs of the
    collision kernel: T, rho_g, c_s, Omega, H, nu_mol, alpha."""
    r_au = np.geomspace(cfg.r_in_au, cfg.r_out_au, cfg.n_r)
    R = r_au * AU
    H = cfg.h_over_r * R
    zfrac = (np.arange(cfg.n_z) + 0.5) / cfg.n_z * cfg.z_max_h
    Rg, Zh = np.meshgrid(R, zfrac, indexing="ij")
    Hg = cfg.h_over_r * Rg
    Z = Zh * Hg
    r_au_g = Rg / AU
    sigma_g = cfg.sigma0 / r_au_g * np.exp(-(5.0 / r_au_g) ** 10)
    rho_g = sigma_g / (np.sqrt(2.0 * np.pi) * Hg) * np.exp(-0.5 * Zh ** 2)
    T = 150.0 * r_au_g ** -0.5
    c_s = np.sqrt(K_B * T / (cfg.mu * M_H))
    Omega = np.sqrt(G_GRAV * M_SUN / (Rg ** 2 + Z ** 2) ** 1.5)
    # molecular viscosity nu_mol = v_th lambda / 2 with lambda = mu m_H / (rho_g sigma_H2)
    v_th = np.sqrt(8.0 / np.pi) * c_s
    lam = cfg.mu * M_H / (rho_g * SIGMA_H2)
    nu_mol = 0.5 * v_th * lam
    if isinstance(cfg.alpha, tuple):
        rng = np.random.default_rng(SEED_ALPHA)
        lo, hi = np.log10(cfg.alpha[0]), np.log10(cfg.alpha[1])
        ring = 10.0 ** rng.uniform(lo, hi, size=cfg.n_r)
        alpha = np.repeat(ring[:, None], cfg.n_z, axis=1)
    else:
        alpha = np.full_like(T, float(cfg.alpha))
    flat = lambda a: np.ascontiguousarray(a.reshape(-1), dtype=np.float64)
    return dict(R=flat(Rg), Z=flat(Z), Sigma_g=flat(sigma_g), T=flat(T), rho_g=flat(rho_g),
                c_s=flat(c_s), Omega=flat(Omega), H=flat(Hg), nu_mol=flat(nu_mol), alpha=flat(alpha))


def make_dust_velocities(cfg: DiscConfig, cells, s):
    """Dust velocities [C][N][3] (v_R, v_phi - v_K, v_Z) in cm/s.

    A stand-in for the dynamics solver: textbook radial drift, azimuthal lag and
    settling driven by the gas pressure gradient of this disc, with the
    midplane Epstein Stokes number (pi/2) rho_m s / Sigma_g raised with height
    as the gas thins.  The azimuthal component is stored relative to the local
    Keplerian speed (relative velocities do not depend on the frame)."""
    R, Z, H = cells["R"], cells["Z"], cells["H"]
    c_s, sig = cells["c_s"], cells["Sigma_g"]
    s = np.asarray(s, dtype=np.float64)
    v_k = np.sqrt(G_GRAV * M_SUN / R)
    r_au = R / AU
    dlnp = -2.5 + 10.0 * (5.0 / r_au) ** 10 + (Z / H) ** 2
    eta = -0.5 * (c_s / v_k) ** 2 * dlnp
    st = (0.5 * np.pi * cfg.rho_m * s[None, :] / sig[:, None]) * np.exp(0.5 * (Z / H)[:, None] ** 2)
    omega_k = v_k / R
    v = np.empty((R.shape[0], s.shape[0], 3))
    v[:, :, 0] = -2.0 * (eta * v_k)[:, None] * st / (1.0 + st ** 2)
    v[:, :, 1] = -(eta * v_k)[:, None] / (1.0 + st ** 2)
    v[:, :, 2] = -(omega_k * Z)[:, None] * st / (1.0 + st ** 2)
    return np.ascontiguousarray(v)


def make_initial_rho(cfg: DiscConfig, cells, s):
    """MRN start: mass per bin ~ s^(1/2) for s <= s_mrn_max, zero above,
    normalised to dust_to_gas * rho_g in every cell.  [C][N] g cm^-3."""
    s = np.asarray(s, dtype=np.float64)
    shape = np.where(s <= cfg.s_mrn_max * (1 + 1e-12), np.sqrt(s), 0.0)
    if not shape.any():             # grid starts above the MRN range: all in bin 0
        shape[0] = 1.0
    shape = shape / shape.sum()
    rho = cfg.dust_to_gas * cells["rho_g"][:, None] * shape[None, :]
    return np.ascontiguousarray(rho)


def make_disc(cfg: DiscConfig, s):
    """Everything one coagulation call needs, for radii s [N] of the bins."""
    cells = make_cells(cfg)
    v = make_dust_velocities(cfg, cells, s)
    rho = make_initial_rho(cfg, cells, s)
    v_frag = np.full(cfg.n_cells, float(cfg.v_frag))
    return dict(cells=cells, v_dust=v, v_frag=v_frag, rho=rho, dt=cfg.dt)


def subset_cells(disc, idx):
    """Cells idx of a disc (same arrays, fewer cells)."""
    idx = np.asarray(idx)
    cells = {k: np.ascontiguousarray(v[idx]) for k, v in disc["cells"].items()}
    return dict(cells=cells, v_dust=np.ascontiguousarray(disc["v_dust"][idx]),
                v_frag=np.ascontiguousarray(disc["v_frag"][idx]),
                rho=np.ascontiguousarray(disc["rho"][idx]), dt=disc["dt"])


# ---------------------------------------------------------------------------
# Vertically integrated columns (surface densities).
# ---------------------------------------------------------------------------
@dataclass
class ColumnConfig:
    """Columns of a disc at n_r radii, each evolved as one cell of the
    vertically integrated kernel: the state is the dust surface density per
    bin, the cell's rho_g the midplane gas density Sigma_g / (sqrt(2 pi) H)
    with H = c_s / Omega.  T = T_ref (R / r_ref)^-1/2; Sigma_g follows the
    disc above, Sigma_0 R_au^-1 exp[-(5/R_au)^10]."""
    name: str
    n_r: int
    n_bins: int
    s_min: float                 # cm
    s_max: float                 # cm
    r_in_au: float = 20.0
    r_out_au: float = 20.0
    T_ref: float = 36.0          # K at r_ref_au
    r_ref_au: float = 20.0
    alpha: float = 1e-3
    v_frag: float = 100.0        # cm/s
    drift: bool = False          # radial drift and azimuthal lag in v_dust (else zero)
    steps: int = 200
    dt: float = 1000.0 * YEAR    # s per coagulation call
    rho_m: float = 1.67
    mu: float = 2.4
    sigma0: float = 250.0
    dust_to_gas: float = 0.01
    s_mrn_max: float = 1.0e-4    # cm

    @property
    def n_cells(self) -> int:
        return self.n_r


COLUMNS = {
    # the paper's single-radius test shape: one column at 20 au, 200 species
    # (0.1 um - 1 m), dynamics off
    "col0d_n200": ColumnConfig("col0d_n200", 1, 200, 1e-5, 100.0),
    # 4096 columns, 5 - 100 au, with radial drift and azimuthal lag
    "col4096_n200": ColumnConfig("col4096_n200", 4096, 200, 1e-5, 100.0, 5.0, 100.0, drift=True),
}


def make_columns(cfg: ColumnConfig, s):
    """Everything one vertically integrated coagulation call needs, for bin
    radii s [N]: per-column gas state (rho_g the midplane density), v_dust
    [C][N][3] (its vertical component unused by that kernel), v_frag, and the
    MRN start as surface densities [C][N] in g cm^-2."""
    r_au = np.geomspace(cfg.r_in_au, cfg.r_out_au, cfg.n_r)
    R = r_au * AU
    T = cfg.T_ref * (r_au / cfg.r_ref_au) ** -0.5
    c_s = np.sqrt(K_B * T / (cfg.mu * M_H))
    Omega = np.sqrt(G_GRAV * M_SUN / R ** 3)
    H = c_s / Omega
    sigma_g = cfg.sigma0 / r_au * np.exp(-(5.0 / r_au) ** 10)
    rho_g = sigma_g / (np.sqrt(2.0 * np.pi) * H)
    v_th = np.sqrt(8.0 / np.pi) * c_s
    nu_mol = 0.5 * v_th * cfg.mu * M_H / (rho_g * SIGMA_H2)
    alpha = np.full(cfg.n_r, float(cfg.alpha))
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    cells = dict(R=f(R), Z=np.zeros(cfg.n_r), Sigma_g=f(sigma_g), T=f(T), rho_g=f(rho_g),
                 c_s=f(c_s), Omega=f(Omega), H=f(H), nu_mol=f(nu_mol), alpha=f(alpha))
    s = np.asarray(s, dtype=np.float64)
    if cfg.drift:
        v = make_dust_velocities(cfg, cells, s)
    else:
        v = np.zeros((cfg.n_r, s.shape[0], 3))
    shape = np.where(s <= cfg.s_mrn_max * (1 + 1e-12), np.sqrt(s), 0.0)
    if not shape.any():
        shape[0] = 1.0
    shape = shape / shape.sum()
    rho = np.ascontiguousarray(cfg.dust_to_gas * sigma_g[:, None] * shape[None, :])
    return dict(cells=cells, v_dust=v, v_frag=np.full(cfg.n_r, float(cfg.v_frag)), rho=rho,
                dt=cfg.dt)


# ---------------------------------------------------------------------------
# Transport inputs: the disc's grid as cylinder and cone faces, gas velocity,
# absolute dust velocities.
# ---------------------------------------------------------------------------
GM_SUN = G_GRAV * M_SUN


def transport_grid(cfg: DiscConfig):
    """Face positions of the disc's cells for the transport step: R_edge
    [n_r + 1] at the geometric midpoints of the log-spaced centres (the end
    faces one half-ratio out), t_edge [n_z + 1] = Z / R of the cone faces, from
    the midplane to z_max_h H / R, so that the cell centres are those of
    make_cells."""
    R = np.geomspace(cfg.r_in_au, cfg.r_out_au, cfg.n_r) * AU
    if cfg.n_r > 1:
        q = np.sqrt(R[1] / R[0])
        R_edge = np.concatenate([[R[0] / q], np.sqrt(R[:-1] * R[1:]), [R[-1] * q]])
    else:
        R_edge = np.array([R[0] / 1.01, R[0] * 1.01])
    t_edge = np.linspace(0.0, cfg.z_max_h * cfg.h_over_r, cfg.n_z + 1)
    return np.ascontiguousarray(R_edge), np.ascontiguousarray(t_edge)


def make_transport(cfg: DiscConfig, s):
    """make_disc plus what the transport step needs: R_edge, t_edge, GM, the
    gas velocity [C][3] (at rest in R and Z, rotating at the sub-Keplerian
    Omega R (1 - eta) of the disc's pressure gradient) and absolute dust
    velocities [C][N][3] (v_phi = the midplane Keplerian speed plus the
    stand-in lag of make_dust_velocities)."""
    d = make_disc(cfg, s)
    cells = d["cells"]
    R, Z, H, c_s = cells["R"], cells["Z"], cells["H"], cells["c_s"]
    v_k = np.sqrt(GM_SUN / R)
    r_au = R / AU
    dlnp = -2.5 + 10.0 * (5.0 / r_au) ** 10 + (Z / H) ** 2
    eta = -0.5 * (c_s / v_k) ** 2 * dlnp
    v_gas = np.zeros((cfg.n_cells, 3))
    v_gas[:, 1] = cells["Omega"] * R * (1.0 - eta)
    v = d["v_dust"].copy()
    v[:, :, 1] += v_k[:, None]
    R_edge, t_edge = transport_grid(cfg)
    d.update(R_edge=R_edge, t_edge=t_edge, GM=GM_SUN, v_gas=np.ascontiguousarray(v_gas),
             v=np.ascontiguousarray(v))
    return d
