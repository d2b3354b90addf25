"""Waves: a batched workload too large for one device, run in pieces.

Every sub-domain's potential is a sum over the sources of its own system
(the multi-domain sum of Sec. II), so the targets of a workload can be
evaluated in any grouping: a plan that evaluates a subset of the targets
(rp_plan_targets) with a split history (each source keeps only the lag
windows of the pairs into those targets) needs far less memory than the
whole system, and its pad covers only its largest target plus the largest
source.  This module groups the targets of every system into units whose
plans fit a memory budget and packs the units into waves, each one batched
plan of several independent unit systems.  Sizes come from the host planner
(no device call); nothing here touches the method's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .plan import Plan


@dataclass
class Unit:
    """Targets `targets` (indices into the workload's domains) of one system,
    with every domain of the system (`domains`) as a source."""
    system: int
    domains: list
    targets: list
    workspace: int = 0
    lagsum_bytes: float = 0.0
    points: int = 0


@dataclass
class Wave:
    units: list = field(default_factory=list)

    @property
    def workspace(self):
        return sum(u.workspace for u in self.units)


def _unit_plan(dims, origins, h, dt, c, precision, local_targets, split_gap, lagsum_steps=1):
    p = Plan(dims, origins, h, dt, c, precision=precision)
    p.set_targets(local_targets)
    if lagsum_steps > 1:
        p.set_tuning("lagsum_steps", lagsum_steps)
    if split_gap > 0:
        p.history_split(split_gap)
    return p


def plan_units(dims, origins, system_id, h, dt, c, precision, budget, split_gap=8, lagsum_steps=1):
    """Units of every system: its targets grouped by grid shape, a group
    halved (along the widest spread of its centres) until its plan fits
    `budget` bytes.  A single target that does not fit raises ValueError."""
    dims = np.asarray(dims, dtype=np.int64).reshape(-1, 3)
    origins = np.asarray(origins, dtype=np.float64).reshape(-1, 3)
    sid = np.zeros(len(dims), dtype=np.int64) if system_id is None else np.asarray(system_id)
    centres = origins + 0.5 * (dims - 1) * h
    units = []
    for k in sorted(set(int(v) for v in sid)):
        doms = [int(i) for i in np.where(sid == k)[0]]
        local = {g: i for i, g in enumerate(doms)}
        shapes = {}
        for g in doms:
            shapes.setdefault(tuple(dims[g]), []).append(g)
        todo = [shapes[key] for key in sorted(shapes)]
        while todo:
            group = todo.pop(0)
            p = _unit_plan(dims[doms], origins[doms], h, dt, c, precision, [local[g] for g in group], split_gap,
                           lagsum_steps)
            ws, st = p.workspace_bytes, p.stats()
            p.close()
            if ws <= budget:
                units.append(Unit(k, doms, list(group), ws, st["lagsum_bytes"], st["points"]))
                continue
            if len(group) == 1:
                raise ValueError(f"target {group[0]} of system {k} alone needs {ws} bytes > budget {budget}")
            spread = centres[group].max(axis=0) - centres[group].min(axis=0)
            axis = int(np.argmax(spread))
            order = sorted(group, key=lambda g: centres[g][axis])
            half = len(order) // 2
            todo[:0] = [order[:half], order[half:]]
    return units


def pack_waves(units, budget):
    """First-fit decreasing packing of the units into waves of at most
    `budget` bytes of summed unit workspace."""
    waves = []
    for u in sorted(units, key=lambda u: -u.workspace):
        for w in waves:
            if w.workspace + u.workspace <= budget:
                w.units.append(u)
                break
        else:
            waves.append(Wave([u]))
    return waves


def wave_layout(wave):
    """Domains of the wave's batched plan: per unit a copy of its system's
    domains with a system id of its own.  Returns (domain indices into the
    workload, system ids, target indices into the wave's domains)."""
    doms, sids, targets = [], [], []
    for ui, u in enumerate(wave.units):
        base = len(doms)
        pos = {g: base + i for i, g in enumerate(u.domains)}
        doms += u.domains
        sids += [ui] * len(u.domains)
        targets += [pos[g] for g in u.targets]
    return doms, sids, targets


def wave_plan(wave, dims, origins, h, dt, c, precision, split_gap=8, stream=None, lagsum_steps=1):
    """The batched plan of one wave (targets set, lag-sum steps per pass,
    history split)."""
    dims = np.asarray(dims).reshape(-1, 3)
    origins = np.asarray(origins).reshape(-1, 3)
    doms, sids, targets = wave_layout(wave)
    p = Plan(dims[doms], origins[doms], h, dt, c, precision=precision, system_id=sids, stream=stream)
    p.set_targets(targets)
    if lagsum_steps > 1:
        p.set_tuning("lagsum_steps", lagsum_steps)
    if split_gap > 0:
        p.history_split(split_gap)
    return p, doms, targets
