"""Seeded synthetic inputs: line lists and pressure-temperature tables.

This module draws random numbers and builds input arrays only; it holds none of
the method's arithmetic.  Both the HIP library and the CPU oracle consume what it
returns.

The paper's workloads are CO2 lines from HITRAN/HITEMP (Section 2.4, Fig. 1:
1 atm, 296 K, 25 cm^-1 cut-off; Section 3.2, Fig. 2: Venus surface, 92.1 bar,
735.3 K, cut-offs 125-500 cm^-1).  Those databases are not available, so the
lists here are synthetic stand-ins with the distributions below, stored with the
precision of the 36-byte database record of Appendix B (wavenumber FP64, every
other field FP32).
"""
from __future__ import annotations

import dataclasses
import struct

import numpy as np

RECORD_BYTES = 36  # Appendix B: 8 (nu) + 7 * 4


@dataclasses.dataclass
class LineList:
    nu0: np.ndarray        # float64 [cm^-1], sorted ascending
    S296: np.ndarray       # float32 [cm/molecule]
    gamma_air: np.ndarray  # float32 [cm^-1/atm]
    gamma_self: np.ndarray # float32 [cm^-1/atm]
    E_lower: np.ndarray    # float32 [cm^-1]
    n_air: np.ndarray      # float32
    mol_iso: np.ndarray    # int32
    delta_air: np.ndarray  # float32 [cm^-1/atm]
    molar_mass: float = 44.0

    @property
    def n(self) -> int:
        return int(self.nu0.shape[0])

    def subset(self, idx) -> "LineList":
        return LineList(*(getattr(self, f.name)[idx] if isinstance(getattr(self, f.name), np.ndarray)
                          else getattr(self, f.name) for f in dataclasses.fields(self)))


def make_lines(n: int, nu_lo: float, nu_hi: float, seed: int, shift: bool = False,
               co2_id: int = 21) -> LineList:
    """n lines, centres U(nu_lo, nu_hi), S296 = 10^U(-26,-19), gamma_air U(0.05,0.1),
    gamma_self = gamma_air, n_air = 0.75, E'' U(0,5000), delta_air U(-0.01,0) if shift."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nu = np.sort(rng.uniform(nu_lo, nu_hi, n))
    S = (10.0 ** rng.uniform(-26.0, -19.0, n)).astype(np.float32)
    g = rng.uniform(0.05, 0.1, n).astype(np.float32)
    E = rng.uniform(0.0, 5000.0, n).astype(np.float32)
    d = (rng.uniform(-0.01, 0.0, n) if shift else np.zeros(n)).astype(np.float32)
    return LineList(nu0=nu.astype(np.float64), S296=S, gamma_air=g, gamma_self=g.copy(),
                    E_lower=E, n_air=np.full(n, 0.75, np.float32),
                    mol_iso=np.full(n, co2_id, np.int32), delta_air=d)


def pt_table(n_layers: int = 100, p_lo: float = 1e-5, p_hi: float = 90.0,
             T_lo: float = 150.0, T_hi: float = 740.0) -> np.ndarray:
    """Layers [n,4] = (p, T, p_self, q_ratio): p log-spaced p_lo..p_hi, T linear
    T_lo..T_hi (hot and dense at the bottom, Venus-like), p_self = p, q_ratio = 0
    (partition ratio 296/T)."""
    i = np.arange(n_layers, dtype=np.float64)
    f = i / max(n_layers - 1, 1)
    p = p_lo * (p_hi / p_lo) ** f
    T = T_lo + (T_hi - T_lo) * f
    return np.stack([p, T, p, np.zeros_like(p)], axis=1)


# workload recipes: synthetic line lists and layers shaped like the paper's workloads
WORKLOADS = {
    # single layer, 1000 lines, Voigt, 25 cm^-1 cut-off, 1000-1010 cm^-1
    "single_1k": dict(lines=(1000, 975.0, 1035.0, 1, False), layers=[(1.0, 296.0, 1.0, 0.0)],
                      nu=(1000.0, 1010.0), cutoff=25.0, chi=0, prune=0.0),
    # single layer, 200k lines, Voigt x Tonkov chi, 125 cm^-1, 500-2500 cm^-1
    "single_200k": dict(lines=(200000, 375.0, 2625.0, 2, True), layers=[(0.1, 250.0, 0.1, 0.0)],
                        nu=(500.0, 2500.0), cutoff=125.0, chi=1, prune=0.0),
    # 100-layer PT table over the same 200k lines, pruned per layer at 1e-10
    "pt100_200k": dict(lines=(200000, 375.0, 2625.0, 2, True), layers="pt100",
                       nu=(500.0, 2500.0), cutoff=125.0, chi=1, prune=1e-10),
    # 100-layer PT table over 2M lines, 0-10000 cm^-1
    "pt100_2m": dict(lines=(2000000, 0.0, 10125.0, 5, True), layers="pt100",
                     nu=(0.0, 10000.0), cutoff=125.0, chi=1, prune=1e-10),
}


def workload(name: str):
    """(LineList, layers[n,4], dict(nu_begin, nu_end, cutoff, chi, prune))."""
    w = WORKLOADS[name]
    n, lo, hi, seed, shift = w["lines"]
    lines = make_lines(n, lo, hi, seed, shift)
    layers = pt_table() if w["layers"] == "pt100" else np.array(w["layers"], np.float64)
    req = dict(nu_begin=w["nu"][0], nu_end=w["nu"][1], cutoff=w["cutoff"], chi=w["chi"],
               prune=w["prune"])
    return lines, layers, req


def pack_records(lines: LineList) -> bytes:
    """Appendix B record layout, little-endian: nu (f8), S, gamma_air, gamma_self,
    E'', n_air (f4), jointMolIso (i4), delta_air (f4)."""
    out = bytearray()
    rec = struct.Struct("<dfffffif")
    for j in range(lines.n):
        out += rec.pack(float(lines.nu0[j]), float(lines.S296[j]), float(lines.gamma_air[j]),
                        float(lines.gamma_self[j]), float(lines.E_lower[j]), float(lines.n_air[j]),
                        int(lines.mol_iso[j]), float(lines.delta_air[j]))
    return bytes(out)


def unpack_records(buf: bytes, molar_mass: float = 44.0) -> LineList:
    dt = np.dtype([("nu", "<f8"), ("S", "<f4"), ("ga", "<f4"), ("gs", "<f4"), ("E", "<f4"),
                   ("n", "<f4"), ("mi", "<i4"), ("d", "<f4")])
    assert dt.itemsize == RECORD_BYTES
    a = np.frombuffer(buf, dtype=dt)
    return LineList(nu0=a["nu"].astype(np.float64), S296=a["S"].copy(), gamma_air=a["ga"].copy(),
                    gamma_self=a["gs"].copy(), E_lower=a["E"].copy(), n_air=a["n"].copy(),
                    mol_iso=a["mi"].copy(), delta_air=a["d"].copy(), molar_mass=molar_mass)
