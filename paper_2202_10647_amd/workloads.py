"""Seeded synthetic inputs: gas level tables, laser fields, initial states.

This module holds no arithmetic of the ionization method itself (no rates, no
chain solution, no window logic).  It only draws inputs, and both the HIP path
and the CPU oracle consume what it returns.

The paper's own workload (krypton in a 9.2 um CO2 laser pulse, Sec. 3 and
Sec. 4) needs measured ionization potentials and the electron structure of its
Fig. 1, which are not reproduced here.  Synthetic level tables with the same
structure stand in for them: Z ionization potentials drawn log-uniformly in a
range and sorted ascending (no rejection of near-equal values, so near-equal
rates occur), with orbital numbers assigned outermost shell first.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

C_LIGHT = 2.99792458e8  # m/s

#: projection code meaning "average the rate over m = -l..l"
M_AVERAGE = -1

# Shell sequences, outermost first: (l, number of electrons).
_SHELLS = {
    7: [(1, 5), (0, 2)],
    18: [(1, 6), (0, 2), (1, 6), (0, 2), (0, 2)],
    36: [(1, 6), (0, 2), (2, 10), (1, 6), (0, 2), (1, 6), (0, 2), (0, 2)],
    54: [(1, 6), (0, 2), (2, 10), (1, 6), (0, 2), (2, 10), (1, 6), (0, 2), (1, 6), (0, 2),
         (0, 2)],
}
_U_RANGE = {1: (13.6, 13.6), 7: (10.0, 700.0), 18: (15.0, 4500.0), 36: (14.0, 18000.0),
            54: (12.0, 41000.0)}
_M_AVG = {36}


@dataclass
class GasTable:
    """U[k] (eV) ionizes charge k -> k+1 with orbital number l[k] and projection
    code m[k] (|m| >= 0, or M_AVERAGE)."""
    name: str
    U: np.ndarray
    l: np.ndarray
    m: np.ndarray

    @property
    def Z(self) -> int:
        return int(self.U.shape[0])


def synthetic_gas(Z: int) -> GasTable:
    """Level table of the synthetic gas with Z levels (Z in 1, 7, 18, 36, 54)."""
    if Z == 1:
        return GasTable("H-like", np.array([13.6]), np.zeros(1, np.int8), np.zeros(1, np.int8))
    lo, hi = _U_RANGE[Z]
    rng = np.random.default_rng(100 + Z)
    U = np.sort(np.exp(rng.uniform(math.log(lo), math.log(hi), size=Z)))
    l = np.concatenate([np.full(n, ll, np.int8) for ll, n in _SHELLS[Z]])
    assert l.shape == (Z,)
    m = np.full(Z, M_AVERAGE if Z in _M_AVG else 0, np.int8)
    return GasTable(f"synthetic-Z{Z}", U, l, m)


def loguniform_field(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """n field values log-uniform in [lo, hi] GV/m (float64)."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))


@dataclass
class LaserMesh:
    """Gaussian laser pulse on a uniform mesh, cell centres, z fastest.
    E(x,z,t) = E0 exp(-(r^2/w0^2 + (z - c t)^2/(c tau)^2)) cos(k0 z - w0 t)."""
    shape: tuple          # (nx, nz) or (nx, ny, nz)
    dx_um: float
    dz_um: float
    E0: float = 3000.0    # GV/m
    lam_um: float = 0.8
    w0_um: float = 20.0
    tau_fs: float = 30.0
    steps: int = 2000

    @property
    def ncells(self) -> int:
        return int(np.prod(self.shape))

    @property
    def dt(self) -> float:
        """0.05 laser periods, in s."""
        return 0.05 * self.lam_um * 1e-6 / C_LIGHT

    def axes_um(self):
        nz = self.shape[-1]
        z = (np.arange(nz) + 0.5) * self.dz_um
        trans = []
        for n in self.shape[:-1]:
            trans.append((np.arange(n) + 0.5 - n / 2) * self.dx_um)
        return trans, z

    def field_at(self, step: int, idx, dtype=np.float64) -> np.ndarray:
        """E at the flat cell indices idx at t = step * dt (float64 arithmetic,
        same formula and operation order as field())."""
        idx = np.asarray(idx, dtype=np.int64)
        trans, z = self.axes_um()
        coords = np.unravel_index(idx, self.shape)
        t = step * self.dt
        ct_um = C_LIGHT * t * 1e6
        k0 = 2 * math.pi / self.lam_um
        om_t = 2 * math.pi * C_LIGHT * t / (self.lam_um * 1e-6)
        r2 = np.zeros(idx.shape)
        for i, a in enumerate(trans):
            r2 = r2 + a[coords[i]] ** 2
        ctau = C_LIGHT * self.tau_fs * 1e-15 * 1e6
        zz = z[coords[-1]]
        env_z = np.exp(-((zz - ct_um) / ctau) ** 2) * np.cos(k0 * zz - om_t)
        return (self.E0 * np.exp(-r2 / self.w0_um ** 2) * env_z).astype(dtype)

    def field(self, step: int, dtype=np.float64) -> np.ndarray:
        """Flat E over all cells at t = step * dt (float64 arithmetic)."""
        trans, z = self.axes_um()
        t = step * self.dt
        ct_um = C_LIGHT * t * 1e6
        k0 = 2 * math.pi / self.lam_um
        om_t = 2 * math.pi * C_LIGHT * t / (self.lam_um * 1e-6)
        r2 = np.zeros([len(a) for a in trans])
        for i, a in enumerate(trans):
            shp = [1] * len(trans)
            shp[i] = a.size
            r2 = r2 + (a.reshape(shp)) ** 2
        ctau = C_LIGHT * self.tau_fs * 1e-15 * 1e6
        env_z = np.exp(-((z - ct_um) / ctau) ** 2) * np.cos(k0 * z - om_t)
        E = self.E0 * np.exp(-r2 / self.w0_um ** 2)[..., None] * env_z
        return E.reshape(-1).astype(dtype)


    def field_torch(self, step: int, device, dtype):
        """field() evaluated with torch on a device (same formula, float64
        arithmetic, cast to dtype); used to keep many steps of E resident in
        device memory without a host round trip."""
        import torch
        trans, z = self.axes_um()
        t = step * self.dt
        ct_um = C_LIGHT * t * 1e6
        k0 = 2 * math.pi / self.lam_um
        om_t = 2 * math.pi * C_LIGHT * t / (self.lam_um * 1e-6)
        ctau = C_LIGHT * self.tau_fs * 1e-15 * 1e6
        zt = torch.from_numpy(z).to(device)
        env_z = torch.exp(-((zt - ct_um) / ctau) ** 2) * torch.cos(k0 * zt - om_t)
        r2 = None
        for i, a in enumerate(trans):
            shp = [1] * len(trans)
            shp[i] = a.size
            term = torch.from_numpy(a).to(device).reshape(shp) ** 2
            r2 = term if r2 is None else r2 + term
        E = self.E0 * torch.exp(-r2 / self.w0_um ** 2)[..., None] * env_z
        return E.reshape(-1).to(dtype)


def mesh_2d() -> LaserMesh:
    """1024 x 1024 2D mesh, 0.08 um cells, E0 = 3000 GV/m, 2000 steps."""
    return LaserMesh((1024, 1024), 0.08, 0.08, E0=3000.0, steps=2000)


def mesh_3d() -> LaserMesh:
    """256 x 256 x 512 3D mesh, 0.32/0.32/0.08 um cells, E0 = 5000 GV/m, 500 steps."""
    return LaserMesh((256, 256, 512), 0.32, 0.08, E0=5000.0, steps=500)


def neutral_state(ncells: int, rows: int, dtype=np.float64):
    """All population in the neutral level: pops[rows][n] with row 0 = 1, lo = 0."""
    pops = np.zeros((rows, ncells), dtype=dtype)
    pops[0] = 1.0
    return pops, np.zeros(ncells, np.uint8)


def random_window_state(ncells: int, Z: int, w: int, seed: int, dtype=np.float64,
                        eps: float = 1e-8):
    """Random normalized window states with varied lowest level lo in [0, Z]:
    compact pops[(w+1)][n].  Slots beyond Z are zero.  Some slots are set
    exactly to zero or below eps so that shifts occur."""
    rng = np.random.default_rng(seed)
    lo = rng.integers(0, Z + 1, size=ncells).astype(np.uint8)
    raw = rng.exponential(size=(w + 1, ncells))
    kill = rng.random((w + 1, ncells))
    raw[kill < 0.2] = 0.0
    raw[(kill >= 0.2) & (kill < 0.3)] *= eps * 0.1
    slot_level = lo[None, :].astype(np.int64) + np.arange(w + 1)[:, None]
    raw[slot_level > Z] = 0.0
    s = raw.sum(axis=0)
    empty = s == 0
    raw[0, empty] = 1.0
    s[empty] = 1.0
    return (raw / s).astype(dtype), lo


# ---------------------------------------------------------------------------
# Mixed gases with uneven windows: a host gas of 1-level cells and a 1 % dopant
# of heavier synthetic gases spread uniformly over the cells.
DOPANT_Z = (7, 18, 36, 54)


def batched_cells(ncells: int, seed: int = 4, dopant_fraction: float = 0.01, wmax: int = 6):
    """(cell_gas, cell_w): gas index 0 is the 1-level gas (w = 1); a Bernoulli
    dopant mask picks cells whose gas is uniform over DOPANT_Z (indices 1..4)
    with w uniform on 1..wmax clamped to Z."""
    rng = np.random.default_rng(seed)
    dop = rng.random(ncells) < dopant_fraction
    gas = np.zeros(ncells, np.uint8)
    w = np.ones(ncells, np.uint8)
    nd = int(dop.sum())
    gi = rng.integers(1, len(DOPANT_Z) + 1, nd).astype(np.uint8)
    zs = np.array((1,) + DOPANT_Z)[gi]
    gas[dop] = gi
    w[dop] = np.minimum(rng.integers(1, wmax + 1, nd), zs).astype(np.uint8)
    return gas, w


_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def hash_field(n: int, seed: int, step: int, E_lo: float = 10.0, E_hi: float = 5000.0, dtype=np.float64):
    """Log-uniform field per (seed, step, cell) from the SplitMix64 finaliser
    (Steele, Lea & Flood 2014) of seed + gamma (step n + i + 1); the same
    definition as the device generator adk_field_hash."""
    with np.errstate(over="ignore"):
        ctr = np.uint64(step) * np.uint64(n) + np.arange(n, dtype=np.uint64) + np.uint64(1)
        z = np.uint64(seed) + _SM_GAMMA * ctr
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    llo = math.log(E_lo)
    return np.exp(llo + u * (math.log(E_hi) - llo)).astype(dtype)


def plan_window_state(cell_gas, cell_w, gas_Z, rows: int, seed: int, fill: float = 0.625, dtype=np.float64):
    """Random window states for a mesh of mixed gases in the plan layout
    pops[rows][n]: each (gas, w) group gets random_window_state draws; rows
    above a cell's window hold `fill` (they must be left untouched)."""
    n = cell_gas.size
    pops = np.full((rows, n), fill, dtype=np.float64)
    lo = np.zeros(n, np.uint8)
    for g, z in enumerate(gas_Z):
        for w in range(1, rows):
            idx = np.nonzero((cell_gas == g) & (cell_w == w))[0]
            if idx.size == 0:
                continue
            comp, l = random_window_state(idx.size, int(z), w, seed=seed + 10 * g + w)
            pops[: w + 1, idx] = comp
            lo[idx] = l
    return pops.astype(dtype), lo


def _splitmix_u01(seed: int, ctr: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the SplitMix64 finaliser of
    seed + gamma * ctr (53 high bits)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + _SM_GAMMA * ctr.astype(np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


#: trained input range of the band-column surrogate: field [GV/m], step [s]
SURROGATE_RANGE = dict(E_lo=10.0, E_hi=5000.0, dt_lo=0.02e-15, dt_hi=0.2e-15)


def surrogate_samples(n: int, seed: int, Z: int, start: int = 0, E_lo: float = 10.0, E_hi: float = 5000.0,
                      dt_lo: float = 0.02e-15, dt_hi: float = 0.2e-15):
    """Training samples start..start+n-1 of the set drawn by `seed`: sample i
    takes three uniforms from counters 3i+1, 3i+2, 3i+3 and maps them to a
    log-uniform field E in [E_lo, E_hi], a log-uniform step dt in
    [dt_lo, dt_hi] and a uniform source level k in 0..Z-1.  The device
    sampler of adk_mlp_train uses the same definition."""
    i = np.arange(start, start + n, dtype=np.uint64)
    u0 = _splitmix_u01(seed, np.uint64(3) * i + np.uint64(1))
    u1 = _splitmix_u01(seed, np.uint64(3) * i + np.uint64(2))
    u2 = _splitmix_u01(seed, np.uint64(3) * i + np.uint64(3))
    lE, lt = math.log(E_lo), math.log(dt_lo)
    E = np.exp(lE + u0 * (math.log(E_hi) - lE))
    dt = np.exp(lt + u1 * (math.log(dt_hi) - lt))
    k = np.minimum(np.floor(u2 * Z), Z - 1).astype(np.int32)
    return E, dt, k


MLP_HIDDEN = 64
MLP_EMB = 16


def mlp_nparams(Z: int) -> int:
    """Flat parameter count: emb[Z][16], W1u[64], W1v[64], W1e[64][16], b1[64],
    W2[64][64], b2[64], W3[64][64], b3[64], W4[4][64], b4[4]."""
    return Z * MLP_EMB + 2 * MLP_HIDDEN + MLP_HIDDEN * MLP_EMB + MLP_HIDDEN + 2 * (MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN) \
        + 4 * MLP_HIDDEN + 4


def mlp_init(Z: int, seed: int = 2022) -> np.ndarray:
    """Seeded initial parameters (float32, flat, in the order above):
    embeddings N(0, 1), weights uniform within +-sqrt(6 / fan_in) (He et al.
    2015), biases zero."""
    rng = np.random.default_rng(seed)
    H, D = MLP_HIDDEN, MLP_EMB
    b0 = math.sqrt(6.0 / (2 + D))
    bh = math.sqrt(6.0 / H)
    parts = [
        rng.standard_normal(Z * D),
        rng.uniform(-b0, b0, H), rng.uniform(-b0, b0, H), rng.uniform(-b0, b0, H * D), np.zeros(H),
        rng.uniform(-bh, bh, H * H), np.zeros(H),
        rng.uniform(-bh, bh, H * H), np.zeros(H),
        rng.uniform(-bh, bh, 4 * H), np.zeros(4),
    ]
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == mlp_nparams(Z)
    return flat
