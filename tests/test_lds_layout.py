"""The bank-aware layout of the packed-rows gathers (host code, lds_layout.h), on the CPU.

* The bank model is pinned to conflict counts measured on the device (SQ_LDS_BANK_CONFLICT per
  8- and 4-byte read instruction, tests/golden/lds_bank_conflicts.json): this file's model, written
  from the measured rules, reproduces every measured count.
* The optimiser only rearranges: its Y cells are a permutation of the species, every physical lane
  holds one input column (same rows, same start slot, same wave), rows keep their class sequence.
* Its reported cycles equal this file's independent evaluation of the model, before and after, and
  the result is deterministic for a seed.
"""
import json
import os
import subprocess
from collections import Counter

import numpy as np
import pytest

from paper_1409_5826_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "lds_bank_conflicts.json")


# ---- bank model, written from the measured rules -------------------------------------------
def half_cycles(addresses):
    """Cycles of one 32-lane half of an 8-byte read: the most distinct addresses on one of the
    64 four-byte banks (an 8-byte address occupies two neighbouring banks)."""
    per_bank = Counter()
    for a in set(int(v) for v in addresses):
        for w in range(2):
            per_bank[(a // 4 + w) % 64] += 1
    return max(per_bank.values())


def instruction_cycles(addresses):
    addresses = list(addresses)
    return sum(half_cycles(addresses[h:h + 32]) for h in range(0, len(addresses), 32))


def half_cycles_b32(addresses):
    """4-byte reads: 32 lanes per half as well, on 32 four-byte banks."""
    per_bank = Counter((a // 4) % 32 for a in set(int(v) for v in addresses))
    return max(per_bank.values())


def instruction_cycles_b32(addresses):
    addresses = list(addresses)
    return sum(half_cycles_b32(addresses[h:h + 32]) for h in range(0, len(addresses), 32))


GENERATORS = {
    "consecutive8": lambda l: 8 * l,
    "broadcast": lambda l: 0,
    "stride16": lambda l: 16 * l,
    "stride128": lambda l: 128 * l,
    "stride256": lambda l: 256 * l,
    "stride512": lambda l: 512 * l,
    "half32_samebanks": lambda l: 8 * (l % 32) + 4096 * (l // 32),
    "quarter16_samebanks": lambda l: 8 * (l % 16) + 4096 * (l // 16),
    "eighth8_samebanks": lambda l: 8 * (l % 8) + 4096 * (l // 8),
    "pairs_samebank": lambda l: 8 * (l // 2) + 4096 * (l % 2),
    "groups_16_32": lambda l: 8 * (l % 32) + 4096 * ((l // 16) % 2),
    "same_addr_pairs": lambda l: 8 * (l // 2),
    "stride8_mod128B": lambda l: 8 * (l % 16),
    "stride8_mod256B": lambda l: 8 * (l % 32),
}

GENERATORS_B32 = {
    "f_consecutive4": lambda l: 4 * l,
    "f_stride8": lambda l: 8 * l,
    "f_stride128": lambda l: 128 * l,
    "f_stride256": lambda l: 256 * l,
    "f_half32_samebanks": lambda l: 4 * (l % 32) + 4096 * (l // 32),
    "f_half32_other": lambda l: 4 * (l % 32) + 128 * (l // 32),
    "f_quarter16_samebanks": lambda l: 4 * (l % 16) + 4096 * (l // 16),
    "f_pairs_samebank": lambda l: 4 * (l // 2) + 4096 * (l % 2),
    "f_lanes_0_32": lambda l: 4 * (l % 64) + (4096 - 128 if l >= 32 else 0),
    "f_broadcast": lambda l: 0,
}


def test_bank_model_reproduces_measured_conflicts():
    g = json.load(open(GOLDEN))
    for case in g["cases"]:
        addr = [GENERATORS[case["pattern"]](l) for l in range(64)]
        assert instruction_cycles(addr) - 2 == case["conflict_cycles"], case["pattern"]
    for case in g["random_cases"]:
        assert instruction_cycles(case["addresses"]) - 2 == case["conflict_cycles"]
    for case in g["cases_b32"]:
        addr = [GENERATORS_B32[case["pattern"]](l) for l in range(64)]
        assert instruction_cycles_b32(addr) - 2 == case["conflict_cycles"], case["pattern"]
    for case in g["random_cases_b32"]:
        assert instruction_cycles_b32(case["addresses"]) - 2 == case["conflict_cycles"]


def test_cells_collide_alike_in_both_precisions():
    # 8-byte cells at 8c and 4-byte cells at 4c conflict exactly when c agrees modulo 32,
    # so one placement serves both precisions
    rng = np.random.default_rng(11)
    for _ in range(200):
        cells = rng.integers(0, 400, 32)
        assert half_cycles(8 * cells) == half_cycles_b32(4 * cells)


# ---- problems ---------------------------------------------------------------------------------
def network_rows(net):
    """Creation and depletion rows as (x, y) species pairs, N = the 1.0 cell."""
    N = net.n_species
    rows = [[] for _ in range(2 * N)]
    for j in range(len(net.product)):
        a, b, c = int(net.reactant0[j]), int(net.reactant1[j]), int(net.product[j])
        rows[c].append((a, b if b >= 0 else N))
        rows[N + a].append((b if b >= 0 else N, N))
        if b >= 0:
            rows[N + b].append((a, N))
    return rows


def make_problem(net, W, seed):
    rng = np.random.default_rng(seed)
    rows = network_rows(net)
    padded = [max(4, (len(r) + 3) // 4 * 4) for r in rows]
    lanes = 64 * W
    load = [0] * lanes
    lane_rows = [[] for _ in range(lanes)]
    for r in sorted(range(len(rows)), key=lambda r: -padded[r]):
        l = int(np.argmin(load))
        lane_rows[l].append(r)
        load[l] += padded[r]
    C = (max(load) + 3) // 4 * 4 + 4
    start = [int(rng.integers(0, (C - load[l]) // 4 + 1)) * 4 for l in range(lanes)]
    cls = [int(v) for v in rng.integers(0, 2, len(rows))]
    return dict(N=net.n_species, lanes=lanes, C=C, rows=rows, padded=padded,
                lane_rows=lane_rows, start=start, cls=cls)


def model_cycles(p, cell_of, lane_rows, start):
    N, C = p["N"], p["C"]
    cell = list(cell_of) + [N]
    xs = np.full((C, p["lanes"]), N)
    ys = np.full((C, p["lanes"]), N)
    for l, rl in enumerate(lane_rows):
        s = start[l]
        for r in rl:
            for e, (x, y) in enumerate(p["rows"][r]):
                xs[s + e, l], ys[s + e, l] = cell[x], cell[y]
            s += p["padded"][r]
    total = 0
    for arr in (xs, ys):
        for s in range(C):
            total += instruction_cycles(8 * arr[s])  # every 32-lane half of every wave
    return total


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("layout") / "driver")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1409_5826_amd", "csrc"),
                    os.path.join(ROOT, "tests", "lds_layout_driver.cpp"), "-o", exe], check=True)
    return exe


def run(driver, p, iters, seed):
    lines = [f"{p['N']} {p['lanes']} {p['C']} {len(p['rows'])} {iters} {seed}"]
    for r, terms in enumerate(p["rows"]):
        lines.append(f"{p['padded'][r]} {len(terms)} " + " ".join(f"{x} {y}" for x, y in terms))
    for l, rl in enumerate(p["lane_rows"]):
        lines.append(f"{p['start'][l]} {len(rl)} " + " ".join(map(str, rl)))
    lines.append(" ".join(map(str, p["cls"])))
    out = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    before, after = map(int, out[0].split())
    cell_of = [int(v) for v in out[1].split()]
    lane_rows, start = [], []
    for l in range(p["lanes"]):
        v = [int(t) for t in out[2 + l].split()]
        start.append(v[0])
        lane_rows.append(v[2:2 + v[1]])
    return before, after, cell_of, lane_rows, start, out


@pytest.mark.parametrize("name,W,seed", [("n16_r48_const", 1, 1), ("n150_r1604_const", 2, 2),
                                         ("n150_r1604_hub_arrhenius", 1, 3)])
def test_layout_rearranges_only_and_reports_its_cost(driver, name, W, seed):
    net = workloads.preset(name, n_zones=1).network
    p = make_problem(net, W, seed)
    before, after, cell_of, lane_rows, start, _ = run(driver, p, 20000, 99 + seed)
    N = p["N"]
    assert sorted(cell_of) == list(range(N))
    # every physical lane holds one input column: same rows in an order, same start, same wave
    cols = {}
    for l, rl in enumerate(p["lane_rows"]):
        cols.setdefault((p["start"][l], tuple(sorted(rl))), []).append(l)
    for l, rl in enumerate(lane_rows):
        key = (start[l], tuple(sorted(rl)))
        assert key in cols and cols[key], f"lane {l} holds no input column"
        src = cols[key].pop()
        assert src // 64 == l // 64, "a column left its wave"
        assert [p["cls"][r] for r in rl] == [p["cls"][r] for r in p["lane_rows"][src]], \
            "rows swapped across classes"
    assert all(not v for v in cols.values())
    # the reported cycles are the model's, before and after
    assert before == model_cycles(p, list(range(N)), p["lane_rows"], p["start"])
    assert after == model_cycles(p, cell_of, lane_rows, start)
    assert after <= before


def test_layout_is_deterministic_and_helps_at_150_species(driver):
    net = workloads.preset("n150_r1604_const", n_zones=1).network
    p = make_problem(net, 2, 7)
    p["start"] = [0] * p["lanes"]
    p["cls"] = [0] * len(p["rows"])
    a = run(driver, p, 30000, 5)
    b = run(driver, p, 30000, 5)
    assert a[5] == b[5]
    before, after = a[0], a[1]
    ideal = 2 * p["C"] * (p["lanes"] // 32)
    assert after < before - 0.3 * (before - ideal), (before, after, ideal)
