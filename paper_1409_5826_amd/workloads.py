"""Seeded synthetic workloads: reaction networks and zone batches.

This module only draws inputs.  It holds none of the integration method's
arithmetic (no fluxes, no sums, no updates, no rate evaluation): the CPU
oracle and the HIP path both consume what it returns, and nothing else is
shared between them.

The paper integrates a 150-species / 1604-reaction thermonuclear network and
shows one of 365 species (section "Implementation of the Explicit Asymptotic
Algorithm on a CPU-GPU System", section "Scaling with Network Size").  Neither
network nor its rate library is available, so these synthetic stand-ins keep
the sizes and the structure the method relies on:

* every species carries an integer weight w_i (its mass number, Eq. 5.35),
  and every reaction conserves weight, so sum_i w_i Y_i is invariant under
  the exact dynamics of Eq. eq1.1;
* one-body reactions A -> B join two distinct species of equal weight;
  two-body reactions A + B -> C join distinct reactants with w_C = w_A + w_B;
* incidence is random, every species takes part in at least `min_incidence`
  reactions, and no reaction appears twice;
* rates are either given per zone (log-uniform constants) or Arrhenius,
  k_j = A_j exp(-E_j / T_z), evaluated by the method itself.

Initial abundances follow X0 ~ Dirichlet(1), Y0 = X0 / w, so that
sum_i w_i Y0_i = 1 (mass fractions summing to one, Eq. 5.35).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Network",
    "Zones",
    "Workload",
    "Schedule",
    "make_schedule",
    "make_network",
    "make_zones",
    "preset",
    "PRESETS",
]


@dataclass
class Network:
    """Reaction structure shared by every zone.

    reactant1[j] == -1 marks a one-body reaction.  A and E are the Arrhenius
    prefactor and activation energy (in units of T) when the rates take that
    form, else None.
    """

    n_species: int
    reactant0: np.ndarray  # int32 [R]
    reactant1: np.ndarray  # int32 [R], -1 for one-body
    product: np.ndarray  # int32 [R]
    weight: np.ndarray  # int32 [N]
    A: Optional[np.ndarray] = None  # float64 [R]
    E: Optional[np.ndarray] = None  # float64 [R]

    @property
    def n_reactions(self) -> int:
        return int(self.reactant0.shape[0])

    @property
    def n_one_body(self) -> int:
        return int(np.count_nonzero(self.reactant1 < 0))

    @property
    def n_two_body(self) -> int:
        return int(np.count_nonzero(self.reactant1 >= 0))

    @property
    def n_destruction(self) -> int:
        """Number of (species, reaction) destruction incidences, R1 + 2 R2."""
        return self.n_one_body + 2 * self.n_two_body

    @property
    def arrhenius(self) -> bool:
        return self.A is not None


@dataclass
class Zones:
    """A batch of independent zones sharing one network.

    Exactly one of T (Arrhenius temperature per zone) and k (rate constants
    per zone and reaction) is set.
    """

    Y0: np.ndarray  # float64 [Z, N]
    t_end: np.ndarray  # float64 [Z]
    dt0: np.ndarray  # float64 [Z]
    T: Optional[np.ndarray] = None  # float64 [Z]
    k: Optional[np.ndarray] = None  # float64 [Z, R]

    @property
    def n_zones(self) -> int:
        return int(self.Y0.shape[0])

    def subset(self, idx) -> "Zones":
        idx = np.asarray(idx)
        return Zones(
            Y0=np.ascontiguousarray(self.Y0[idx]),
            t_end=np.ascontiguousarray(self.t_end[idx]),
            dt0=np.ascontiguousarray(self.dt0[idx]),
            T=None if self.T is None else np.ascontiguousarray(self.T[idx]),
            k=None if self.k is None else np.ascontiguousarray(self.k[idx]),
        )


@dataclass
class Workload:
    name: str
    network: Network
    zones: Zones
    tol: float
    description: str
    extra: dict = field(default_factory=dict)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _candidates(weight: np.ndarray):
    """All admissible reactions for the weights: (one-body pairs, two-body triples)."""
    n = weight.shape[0]
    one = [(a, b) for a in range(n) for b in range(n) if a != b and weight[a] == weight[b]]
    by_w: dict[int, list[int]] = {}
    for i in range(n):
        by_w.setdefault(int(weight[i]), []).append(i)
    two = []
    for a in range(n):
        for b in range(a + 1, n):
            for c in by_w.get(int(weight[a] + weight[b]), ()):
                two.append((a, b, c))
    return np.array(one, dtype=np.int64).reshape(-1, 2), np.array(two, dtype=np.int64).reshape(-1, 3)


def make_network(
    n_species: int,
    n_one_body: int,
    n_two_body: int,
    mass_group: int,
    seed: int,
    min_incidence: int = 4,
    arrhenius: Optional[tuple[float, float, float, float]] = None,
    hubs: tuple = (),
    hub_fraction: float = 0.0,
) -> Network:
    """Draw a weight-conserving random network.

    mass_group species share each weight: w_i = 1 + floor(i / mass_group).
    arrhenius = (log10A_lo, log10A_hi, E_lo, E_hi) draws log10 A_j ~ U(log10A_lo,
    log10A_hi) and E_j ~ U(E_lo, E_hi); None leaves rates to the zones.
    hubs / hub_fraction: that fraction of the two-body reactions drawn after the
    coverage phase has a hub species as a reactant (light particles captured by
    everything, as protons, neutrons and alpha particles are in nuclear networks).
    """
    rng = _rng(seed)
    weight = (1 + np.arange(n_species) // mass_group).astype(np.int32)
    one, two = _candidates(weight)
    if n_one_body > len(one) or n_two_body > len(two):
        raise ValueError("not enough admissible reactions for the requested counts")
    # incidence lists of the candidates, for the coverage phase
    one_of = [[] for _ in range(n_species)]
    for idx, (a, b) in enumerate(one):
        one_of[a].append(idx)
        one_of[b].append(idx)
    two_of = [[] for _ in range(n_species)]
    for idx, (a, b, c) in enumerate(two):
        two_of[a].append(idx)
        two_of[b].append(idx)
        two_of[c].append(idx)
    used1 = np.zeros(len(one), dtype=bool)
    used2 = np.zeros(len(two), dtype=bool)
    inc = np.zeros(n_species, dtype=np.int64)
    n1 = n2 = 0

    def take1(idx):
        nonlocal n1
        used1[idx] = True
        n1 += 1
        inc[one[idx, 0]] += 1
        inc[one[idx, 1]] += 1

    def take2(idx):
        nonlocal n2
        used2[idx] = True
        n2 += 1
        for s in two[idx]:
            inc[s] += 1

    # coverage: every species takes part in at least min_incidence reactions
    for s in rng.permutation(n_species):
        while inc[s] < min_incidence:
            rem1, rem2 = n_one_body - n1, n_two_body - n2
            if rem1 + rem2 <= 0:
                raise ValueError("reaction budget too small for the incidence floor")
            free1 = [i for i in one_of[s] if not used1[i]] if rem1 > 0 else []
            free2 = [i for i in two_of[s] if not used2[i]] if rem2 > 0 else []
            if not free1 and not free2:
                raise ValueError(f"species {s} cannot reach the incidence floor")
            pick_one = bool(free1) and (not free2 or rng.random() < rem1 / (rem1 + rem2))
            if pick_one:
                take1(free1[int(rng.integers(len(free1)))])
            else:
                take2(free2[int(rng.integers(len(free2)))])
    # fill the remaining budget uniformly from the unused candidates
    rest1 = np.flatnonzero(~used1)
    for idx in rng.choice(rest1, size=n_one_body - n1, replace=False):
        take1(int(idx))
    rest2 = np.flatnonzero(~used2)
    left2 = n_two_body - n2
    if hubs and hub_fraction > 0.0:
        hub = np.isin(two[:, 0], hubs) | np.isin(two[:, 1], hubs)
        rest_hub, rest_other = rest2[hub[rest2]], rest2[~hub[rest2]]
        n_hub = min(len(rest_hub), int(round(hub_fraction * left2)))
        picks = np.concatenate([rng.choice(rest_hub, size=n_hub, replace=False),
                                rng.choice(rest_other, size=left2 - n_hub, replace=False)])
    else:
        picks = rng.choice(rest2, size=left2, replace=False)
    for idx in picks:
        take2(int(idx))

    sel1 = one[used1]
    sel2 = two[used2]
    r0 = np.concatenate([sel1[:, 0], sel2[:, 0]])
    r1 = np.concatenate([np.full(len(sel1), -1), sel2[:, 1]])
    pr = np.concatenate([sel1[:, 1], sel2[:, 2]])
    # random reaction order, and a random reactant order within two-body reactions
    perm = rng.permutation(len(r0))
    r0, r1, pr = r0[perm], r1[perm], pr[perm]
    swap = (r1 >= 0) & (rng.random(len(r0)) < 0.5)
    r0[swap], r1[swap] = r1[swap], r0[swap].copy()
    net = Network(
        n_species=n_species,
        reactant0=r0.astype(np.int32),
        reactant1=r1.astype(np.int32),
        product=pr.astype(np.int32),
        weight=weight,
    )
    if arrhenius is not None:
        lo, hi, e_lo, e_hi = arrhenius
        log10_a = rng.uniform(lo, hi, size=net.n_reactions)
        net.A = np.power(10.0, log10_a)
        net.E = rng.uniform(e_lo, e_hi, size=net.n_reactions)
    return net


def make_zones(
    net: Network,
    n_zones: int,
    seed: int,
    t_end: float,
    dt0: float = 1e-12,
    log10_k_range: Optional[tuple[float, float]] = None,
    T_range: Optional[tuple[float, float]] = None,
) -> Zones:
    """Draw per-zone initial abundances and either constant rates or temperatures.

    Y0: X0 ~ Dirichlet(1_N), Y0 = X0 / w.  log10_k_range draws log10 k_zj
    uniformly (constant rates); T_range draws T_z log-uniformly (Arrhenius).
    """
    rng = _rng(seed)
    n = net.n_species
    x0 = rng.dirichlet(np.ones(n), size=n_zones)
    y0 = x0 / net.weight.astype(np.float64)[None, :]
    z = Zones(
        Y0=np.ascontiguousarray(y0),
        t_end=np.full(n_zones, float(t_end)),
        dt0=np.full(n_zones, float(dt0)),
    )
    if log10_k_range is not None:
        lo, hi = log10_k_range
        z.k = np.ascontiguousarray(np.power(10.0, rng.uniform(lo, hi, size=(n_zones, net.n_reactions))))
    if T_range is not None:
        lo, hi = T_range
        z.T = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_zones))
    if (z.k is None) == (z.T is None):
        raise ValueError("give exactly one of log10_k_range and T_range")
    return z


# Activation-energy windows of the Arrhenius workloads, in units of T.  Each
# was chosen with the oracle (a calibration sweep run once) so that accepted
# step counts over zones with T log-uniform in [1, 4] spread by about 10x
# between the 10th and the 90th percentile (10.5x over 128 zones of the
# 150-species network, 11.2x over 64 zones of the 365-species one).  A window
# starting at 0 leaves every zone with a broad set of fast reactions and a
# spread of only about 1.5x.
ARRHENIUS_E_WINDOW_N150 = (27.5, 90.0)
ARRHENIUS_E_WINDOW_N365 = (30.0, 90.0)


def _n16(n_zones=1):
    net = make_network(16, 24, 24, mass_group=4, seed=1001)
    zones = make_zones(net, n_zones, seed=2001, t_end=1e-2, log10_k_range=(-4.0, 8.0))
    return Workload("n16_r48_const", net, zones, 0.01,
                    "16 species, 48 reactions (24 one-body, 24 two-body), constant rates "
                    "log-uniform 1e-4..1e8, single zone, t_end 1e-2 s")


def _n150_const(n_zones=128, seed_offset=0):
    net = make_network(150, 481, 1123, mass_group=5, seed=1002)
    zones = make_zones(net, n_zones, seed=2002 + seed_offset, t_end=1.0, log10_k_range=(-6.0, 10.0))
    return Workload("n150_r1604_const", net, zones, 0.01,
                    "150 species, 1604 reactions (481 one-body, 1123 two-body), constant per-zone "
                    "rates log-uniform 1e-6..1e10, t_end 1 s")


def _n150_arrh(n_zones=4096, e_window=None):
    e_lo, e_hi = ARRHENIUS_E_WINDOW_N150 if e_window is None else e_window
    net = make_network(150, 481, 1123, mass_group=5, seed=1003, arrhenius=(2.0, 12.0, e_lo, e_hi))
    zones = make_zones(net, n_zones, seed=2003, t_end=1.0, T_range=(1.0, 4.0))
    return Workload("n150_r1604_arrhenius", net, zones, 0.01,
                    "150 species, 1604 reactions, Arrhenius rates (log10 A in 2..12, "
                    f"E in {e_lo:g}..{e_hi:g}), T log-uniform 1..4 per zone, t_end 1 s",
                    extra={"E_window": (e_lo, e_hi)})


def _n150_hub(n_zones=4096, e_window=None):
    e_lo, e_hi = ARRHENIUS_E_WINDOW_N150 if e_window is None else e_window
    net = make_network(150, 481, 1123, mass_group=5, seed=1005, arrhenius=(2.0, 12.0, e_lo, e_hi),
                       hubs=(0, 1, 15), hub_fraction=0.6)
    zones = make_zones(net, n_zones, seed=2005, t_end=1.0, T_range=(1.0, 4.0))
    return Workload("n150_r1604_hub_arrhenius", net, zones, 0.01,
                    "150 species, 1604 reactions, 60 % of the freely drawn two-body reactions "
                    "capture one of 3 hub species (weights 1, 1, 4), Arrhenius rates as the "
                    "150-species workload, T log-uniform 1..4 per zone, t_end 1 s",
                    extra={"E_window": (e_lo, e_hi), "hubs": (0, 1, 15)})


def _n365_arrh(n_zones=1024, e_window=None):
    e_lo, e_hi = ARRHENIUS_E_WINDOW_N365 if e_window is None else e_window
    net = make_network(365, 1320, 3080, mass_group=6, seed=1004, arrhenius=(2.0, 12.0, e_lo, e_hi))
    zones = make_zones(net, n_zones, seed=2004, t_end=1.0, T_range=(1.0, 4.0))
    return Workload("n365_r4400_arrhenius", net, zones, 0.01,
                    "365 species, 4400 reactions (1320 one-body, 3080 two-body), Arrhenius rates "
                    f"(log10 A in 2..12, E in {e_lo:g}..{e_hi:g}), T log-uniform 1..4 per zone, "
                    "t_end 1 s",
                    extra={"E_window": (e_lo, e_hi)})


@dataclass
class Schedule:
    """Inputs of an operator-split sequence of hydro steps for a batch of zones."""

    T: Optional[np.ndarray]   # float64 [n_steps, Z] temperature per step (Arrhenius zones)
    dt_hydro: np.ndarray      # float64 [n_steps, Z] interval of each step
    q: np.ndarray             # float64 [N] energy per unit abundance of each species

    @property
    def n_steps(self) -> int:
        return int(self.dt_hydro.shape[0])


def make_schedule(net: Network, zones: Zones, n_steps: int, seed: int,
                  T_swing: float = 0.1) -> Schedule:
    """Split each zone's interval into n_steps equal hydro steps; Arrhenius zones get a
    temperature path T_z (1 + T_swing sin(2 pi (s / n_steps + phase_z))), seeded phases; the
    energy coefficients are a smooth function of the weight, q_i = w_i (8 - 9 w_i^(-1/3)),
    plus 1 % seeded noise."""
    rng = _rng(seed)
    Z = zones.n_zones
    dt_h = np.tile(zones.t_end / n_steps, (n_steps, 1))
    T = None
    if zones.T is not None:
        phase = rng.uniform(0.0, 1.0, size=Z)
        s = np.arange(n_steps)[:, None]
        T = zones.T[None, :] * (1.0 + T_swing * np.sin(2.0 * np.pi * (s / n_steps + phase[None, :])))
    w = net.weight.astype(np.float64)
    q = w * (8.0 - 9.0 * w ** (-1.0 / 3.0)) * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=net.n_species))
    return Schedule(T=None if T is None else np.ascontiguousarray(T),
                    dt_hydro=np.ascontiguousarray(dt_h), q=np.ascontiguousarray(q))


PRESETS = {
    "n16_r48_const": _n16,
    "n150_r1604_const": _n150_const,
    "n150_r1604_arrhenius": _n150_arrh,
    "n365_r4400_arrhenius": _n365_arrh,
    "n150_r1604_hub_arrhenius": _n150_hub,
}


def preset(name: str, n_zones: Optional[int] = None, **kw) -> Workload:
    """Build a named workload; n_zones overrides the preset's zone count."""
    fn = PRESETS[name]
    if n_zones is not None:
        kw["n_zones"] = n_zones
    return fn(**kw)
