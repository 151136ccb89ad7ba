"""Container for one instance of the epidemic problem statement.

The fields follow the paper's statement of the problem (arXiv:1502.02908):
the integer compartment matrix X (Sec. 2.2, stored node-major as the paper's
columns X^(i)), the continuous state Y (Sec. 2.3; here one row, the
environmental infectious pressure phi), the stoichiometry S of the stochastic
transitions (Sec. 2.1), the propensity description of Sec. 3.3 / eq:rate_s_to_i
/ eq:recovery_rates, the phi model of eq:siminfpressure, and the day-sorted
external event list of Sec. 3.2 (eq:event) extended by a select matrix E (which
compartments an event draws from) and a shift matrix N (where a moved
individual lands, relative to its compartment).

This module holds data only: no step of the method is computed here.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Optional

import numpy as np

EXIT, ENTER, INTERNAL, EXTERNAL = 0, 1, 2, 3
KIND_NAMES = {EXIT: "exit", ENTER: "enter", INTERNAL: "internal", EXTERNAL: "external"}


@dataclasses.dataclass
class Problem:
    n_nodes: int
    n_comp: int
    n_trans: int
    n_rep: int
    n_days: int
    u0: np.ndarray            # int32 [Nn, Nc]
    v0: np.ndarray            # float64 [Nn]
    S: np.ndarray             # int32 [Nc, Nt]
    reactant: np.ndarray      # int32 [Nt]
    uses_phi: np.ndarray      # int32 [Nt]
    coef: np.ndarray          # float64 [R, Nt]
    alpha: np.ndarray         # float64 [R]
    beta: np.ndarray          # float64 [R, 4]
    phi_I_mask: int
    phi_N_mask: int
    E: np.ndarray             # int32 [Nc, n_select]
    N: np.ndarray             # int32 [Nc, n_shift]
    ev_day: np.ndarray        # int32 [n_events], ascending
    ev_kind: np.ndarray       # int32
    ev_node: np.ndarray       # int32
    ev_dest: np.ndarray       # int32 (-1 for single-node events)
    ev_n: np.ndarray          # int32
    ev_select: np.ndarray     # int32
    ev_shift: np.ndarray      # int32 (-1 = no shift)
    seed: int = 1
    day0: int = 0
    replicate_id: Optional[np.ndarray] = None  # uint32 [R]
    reactant2: Optional[np.ndarray] = None  # int32 [Nt]: second reactant of a mass-action rate, -1 none
    phi_pre_events: int = 0  # 1: phi is fed by the state before the day's events
    n_regions: int = 0       # regions of the goal function's aggregates (Sec. 4.3)
    region: Optional[np.ndarray] = None  # int32 [Nn] region of each node, or -1
    record_days: Optional[np.ndarray] = None   # int32 ascending
    name: str = ""

    def __post_init__(self):
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.u0 = i32(self.u0).reshape(self.n_nodes, self.n_comp)
        self.v0 = f64(self.v0).reshape(self.n_nodes)
        self.S = i32(self.S).reshape(self.n_comp, self.n_trans)
        self.reactant = i32(self.reactant)
        self.uses_phi = i32(self.uses_phi)
        self.coef = f64(self.coef).reshape(self.n_rep, self.n_trans)
        self.alpha = f64(self.alpha).reshape(self.n_rep)
        self.beta = f64(self.beta).reshape(self.n_rep, 4)
        self.E = i32(self.E).reshape(self.n_comp, -1)
        self.N = i32(self.N).reshape(self.n_comp, -1)
        for f in ("ev_day", "ev_kind", "ev_node", "ev_dest", "ev_n", "ev_select", "ev_shift"):
            setattr(self, f, i32(getattr(self, f)))
        if self.replicate_id is None:
            self.replicate_id = np.arange(self.n_rep, dtype=np.uint32)
        self.replicate_id = np.ascontiguousarray(self.replicate_id, dtype=np.uint32)
        if self.reactant2 is not None:
            self.reactant2 = i32(self.reactant2)
        if self.region is not None:
            self.region = i32(self.region).reshape(self.n_nodes)
        if self.record_days is None:
            self.record_days = np.zeros(0, dtype=np.int32)
        self.record_days = i32(self.record_days)

    @property
    def n_events(self) -> int:
        return int(self.ev_day.shape[0])

    @property
    def n_select(self) -> int:
        return int(self.E.shape[1])

    @property
    def n_shift(self) -> int:
        return int(self.N.shape[1])

    def with_replicates(self, R: int, coef=None, alpha=None, beta=None, replicate_id=None) -> "Problem":
        """Same network and events, R replicates; parameters broadcast unless given."""
        coef = np.broadcast_to(self.coef[0], (R, self.n_trans)) if coef is None else coef
        alpha = np.broadcast_to(self.alpha[0], (R,)) if alpha is None else alpha
        beta = np.broadcast_to(self.beta[0], (R, 4)) if beta is None else beta
        return dataclasses.replace(self, n_rep=R, coef=np.array(coef), alpha=np.array(alpha),
                                   beta=np.array(beta), replicate_id=replicate_id)

    def truncated(self, n_days: int) -> "Problem":
        """The same problem with a shorter horizon (events past it dropped)."""
        keep = self.ev_day < n_days
        kw = {f: getattr(self, f)[keep] for f in
              ("ev_day", "ev_kind", "ev_node", "ev_dest", "ev_n", "ev_select", "ev_shift")}
        rec = self.record_days[self.record_days < n_days]
        return dataclasses.replace(self, n_days=n_days, record_days=rec, **kw)

    def digest(self) -> str:
        h = hashlib.sha256()
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            if isinstance(v, np.ndarray):
                h.update(f.name.encode()); h.update(np.ascontiguousarray(v).tobytes())
            else:
                h.update(f"{f.name}={v!r}".encode())
        return h.hexdigest()[:16]

    def event_counts(self):
        return {KIND_NAMES[k]: int((self.ev_kind == k).sum()) for k in KIND_NAMES}
