"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module only draws random numbers and lays out circuit descriptions; it
holds none of the simulation arithmetic (no gate matrices for named gates, no
state updates, no expectation values).  Both sides turn a :class:`Gate` into a
matrix with their own code.

Circuit conventions follow the paper (Sec. III): qubit 0 is the least
significant index bit, a gate is a single-qubit operation on ``target`` with
any number of ``controls``.  ``values`` gives the required value of each
control (the paper uses value 1 only; the negative-control identity of the
two-qubit circuit figure in Sec. I motivates value 0).

Workloads (all seeded, all synthetic):

* ``random_gates_n12``  n=12, 200 gates from {X, H, RY, RZ}, 0-3 controls.
* ``gate_sweep_*``     n=28 random normalised state, one Haar 2x2, target in
  {0, 13, 27}, c = 0..8 controls on random distinct qubits.
* ``layered_circuit_n32`` n=32, 20 layers of (H or RY on every qubit, CNOT ladder,
  8 multi-controlled X with 1-6 controls).
* ``hea_problem_n24``  n=24 hardware-efficient ansatz, 16 layers of RY, RZ on every
  qubit plus a CNOT chain (768 parameters); H = sum a_i Z_i Z_{i+1} + b_i X_i.
* ``uneven_batch``     4096 circuits with n uniform in 10..20 and 100-400 gates as in
  random_gates_n12; plus 256 ansatz circuits at n=16 with 4 layers for batched
  gradients.
* the paper's own evaluation circuits: the QFT staircase (Sec. IV-A figure)
  and the streaming circuit (Sec. IV-C figure).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi

# Gate kinds understood by both sides.  "U" carries an explicit matrix drawn
# here (a random unitary is an input, not part of the method).
KINDS = ("X", "Y", "Z", "H", "RX", "RY", "RZ", "P", "U")
PARAM_KINDS = ("RX", "RY", "RZ", "P")


@dataclass(frozen=True)
class Gate:
    kind: str
    target: int
    controls: Tuple[int, ...] = ()
    values: Tuple[int, ...] = ()          # aligned with controls; empty = all 1
    theta: float = 0.0                    # angle of RX/RY/RZ/P when param < 0
    param: int = -1                       # index into a parameter vector
    matrix: Optional[Tuple[float, ...]] = None  # 8 floats, kind "U" only

    def control_values(self) -> Tuple[int, ...]:
        return self.values if self.values else tuple(1 for _ in self.controls)

    def qubits(self) -> Tuple[int, ...]:
        return (self.target,) + tuple(self.controls)


@dataclass(frozen=True)
class PauliTerm:
    """coef * i^{|x&z|} X^x Z^z; bit q of x (z) places X (Z) on qubit q."""
    coef: float
    x_mask: int
    z_mask: int


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    params: Optional[np.ndarray] = None   # values for gates with param >= 0
    meta: dict = field(default_factory=dict)

    @property
    def nparams(self) -> int:
        return 0 if self.params is None else int(len(self.params))


# --------------------------------------------------------------------------
# serialised circuit format (JSON): one object per circuit
#   {"n": n, "gates": [[kind, target, [controls], [values], theta, param,
#                       matrix-or-null], ...], "params": [...] or null,
#    "meta": {...}}
# Floats are written with repr precision, so a round trip is exact.
# --------------------------------------------------------------------------

def circuit_to_json(c: Circuit) -> dict:
    return {"n": int(c.n),
            "gates": [[g.kind, int(g.target), [int(q) for q in g.controls], [int(v) for v in g.values],
                       float(g.theta), int(g.param), None if g.matrix is None else [float(x) for x in g.matrix]]
                      for g in c.gates],
            "params": None if c.params is None else [float(x) for x in c.params],
            "meta": dict(c.meta)}


def circuit_from_json(d: dict) -> Circuit:
    gates = [Gate(k, int(t), tuple(int(q) for q in cs), tuple(int(v) for v in vs), float(th), int(p),
                  None if m is None else tuple(float(x) for x in m))
             for k, t, cs, vs, th, p, m in d["gates"]]
    params = None if d.get("params") is None else np.asarray(d["params"], dtype=np.float64)
    return Circuit(int(d["n"]), gates, params, dict(d.get("meta") or {}))


def save_circuits(path: str, circuits: Sequence[Circuit]) -> None:
    """One JSON object per line."""
    import json
    with open(path, "w") as f:
        for c in circuits:
            f.write(json.dumps(circuit_to_json(c)) + "\n")


def load_circuits(path: str) -> List[Circuit]:
    import json
    with open(path) as f:
        return [circuit_from_json(json.loads(line)) for line in f if line.strip()]


# --------------------------------------------------------------------------
# random primitives
# --------------------------------------------------------------------------

def random_state(n: int, seed: int) -> np.ndarray:
    """Real and imaginary parts i.i.d. N(0,1), then scaled to unit norm."""
    rng = np.random.default_rng(seed)
    dim = 1 << n
    v = np.empty(dim, dtype=np.complex128)
    f = v.view(np.float64)
    # fill in chunks to bound peak memory for large n
    chunk = 1 << 24
    for s in range(0, 2 * dim, chunk):
        e = min(2 * dim, s + chunk)
        f[s:e] = rng.standard_normal(e - s)
    nrm = np.sqrt(np.vdot(v, v).real)
    v /= nrm
    return v


def haar_unitary_2x2(seed: int) -> Tuple[float, ...]:
    """Haar-distributed 2x2 unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q (Mezzadri, Notices AMS 2007).
    Returned as 8 floats, row-major (re, im) pairs."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    q = q * (d / np.abs(d))
    return tuple(float(v) for c in q.reshape(-1) for v in (c.real, c.imag))


def _random_controlled_gates(rng: np.random.Generator, n: int, ngates: int,
                             max_controls: int = 3) -> List[Gate]:
    """Random controlled gates.  Per gate the draw order is fixed: kind, then the
    angle (RY/RZ only), target, number of controls, controls."""
    kinds = ("X", "H", "RY", "RZ")
    out = []
    for _ in range(ngates):
        kind = kinds[int(rng.integers(0, 4))]
        theta = float(rng.uniform(0.0, TWO_PI)) if kind in ("RY", "RZ") else 0.0
        t = int(rng.integers(0, n))
        nc = int(rng.integers(0, min(max_controls, n - 1) + 1))
        others = [q for q in range(n) if q != t]
        ctrls = tuple(int(q) for q in rng.choice(others, size=nc, replace=False)) if nc else ()
        out.append(Gate(kind, t, ctrls, (), theta))
    return out


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def random_gates_n12(seed: int = 0, n: int = 12, ngates: int = 200) -> Circuit:
    rng = np.random.default_rng(seed)
    return Circuit(n, _random_controlled_gates(rng, n, ngates),
                   meta={"name": "random_gates_n12", "seed": seed})


SWEEP_TARGETS = (0, 13, 27)
SWEEP_CONTROLS = tuple(range(0, 9))


def gate_sweep_cases(n: int = 28, seed: int = 3,
                  targets: Sequence[int] = SWEEP_TARGETS,
                  counts: Sequence[int] = SWEEP_CONTROLS):
    """(target, controls) for every target and control count, controls drawn
    as random distinct qubits other than the target.  Draw order: for each
    target in order, for each count in order, the controls."""
    rng = np.random.default_rng(seed)
    cases = []
    for t in targets:
        others = [q for q in range(n) if q != t]
        for c in counts:
            ctrls = tuple(sorted(int(q) for q in rng.choice(others, size=c, replace=False))) if c else ()
            cases.append((int(t), ctrls))
    return cases


def sweep_unitary(seed: int = 2) -> Tuple[float, ...]:
    return haar_unitary_2x2(seed)


def layered_circuit_n32(seed: int = 4, n: int = 32, layers: int = 20, mcx_per_layer: int = 8,
            mcx_controls: Tuple[int, int] = (1, 6)) -> Circuit:
    """Per layer: H or RY(theta) (fair coin per qubit) on every qubit, a CNOT
    ladder (control i, target i+1), then multi-controlled X gates with a
    uniform number of random controls."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(layers):
        for q in range(n):
            if rng.integers(0, 2) == 0:
                gates.append(Gate("H", q))
            else:
                gates.append(Gate("RY", q, theta=float(rng.uniform(0.0, TWO_PI))))
        for q in range(n - 1):
            gates.append(Gate("X", q + 1, (q,)))
        for _ in range(mcx_per_layer):
            t = int(rng.integers(0, n))
            nc = int(rng.integers(mcx_controls[0], mcx_controls[1] + 1))
            others = [q for q in range(n) if q != t]
            ctrls = tuple(int(q) for q in rng.choice(others, size=nc, replace=False))
            gates.append(Gate("X", t, ctrls))
    return Circuit(n, gates, meta={"name": "layered_n32", "seed": seed})


def hea(n: int, layers: int, seed: int) -> Circuit:
    """Hardware-efficient ansatz: per layer RY(theta) then RZ(theta) on every
    qubit, then a CNOT chain (control i, target i+1).  Parameters are numbered
    in gate order; theta ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    p = 0
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate("RY", q, param=p)); p += 1
            gates.append(Gate("RZ", q, param=p)); p += 1
        for q in range(n - 1):
            gates.append(Gate("X", q + 1, (q,)))
    params = rng.uniform(0.0, TWO_PI, size=p)
    return Circuit(n, gates, params, meta={"name": "hea", "seed": seed})


def zz_x_hamiltonian(n: int, seed: int) -> List[PauliTerm]:
    """H = sum_{i=0}^{n-2} a_i Z_i Z_{i+1} + sum_{i=0}^{n-1} b_i X_i (open
    chain), a_i, b_i ~ N(0,1); a drawn first, then b."""
    rng = np.random.default_rng(seed + 1000)
    a = rng.standard_normal(n - 1)
    b = rng.standard_normal(n)
    terms = [PauliTerm(float(a[i]), 0, (1 << i) | (1 << (i + 1))) for i in range(n - 1)]
    terms += [PauliTerm(float(b[i]), 1 << i, 0) for i in range(n)]
    return terms


def hea_problem_n24(seed: int = 5, n: int = 24, layers: int = 16):
    c = hea(n, layers, seed)
    c.meta["name"] = "hea_n24"
    return c, zz_x_hamiltonian(n, seed)


def uneven_batch(seed: int = 6, ncirc: int = 4096, nrange=(10, 20), grange=(100, 400)) -> List[Circuit]:
    """Independent circuits of uneven width; per circuit draw n, then the gate
    count, then the gates as in random_gates_n12."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(ncirc):
        n = int(rng.integers(nrange[0], nrange[1] + 1))
        g = int(rng.integers(grange[0], grange[1] + 1))
        out.append(Circuit(n, _random_controlled_gates(rng, n, g), meta={"index": i}))
    return out


def low_control_circuit(n: int = 28, ngates: int = 24, seed: int = 9) -> Circuit:
    """Gates whose controls sit mostly on the lowest qubits (below the
    128-byte granule of a complex128 state): per gate, kind uniform in
    {X, H, RY}, target uniform in 3..n-1, one or two controls from {0, 1, 2}
    and, with probability 1/2, one more control uniform among the other
    qubits (value 1 throughout)."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(ngates):
        kind = ("X", "H", "RY")[int(rng.integers(0, 3))]
        t = int(rng.integers(3, n))
        k = int(rng.integers(1, 3))
        ctrls = [int(q) for q in rng.choice(3, size=k, replace=False)]
        if rng.random() < 0.5:
            others = [q for q in range(3, n) if q != t]
            ctrls.append(int(rng.choice(others)))
        theta = float(rng.uniform(0, TWO_PI)) if kind == "RY" else 0.0
        gates.append(Gate(kind, t, tuple(sorted(ctrls)), (), theta))
    return Circuit(n, gates, meta={"name": "low_control", "seed": seed})


def hea_batch_n16(seed: int = 7, ncirc: int = 256, n: int = 16, layers: int = 4):
    """Batched-gradient workload: the n=24 problem's ansatz at n=16 with 4 layers
    (128 parameters) per circuit, each circuit with its own angles and its own
    ZZ+X Hamiltonian."""
    out = []
    for i in range(ncirc):
        c = hea(n, layers, seed * 100003 + i)
        out.append((c, zz_x_hamiltonian(n, seed * 100003 + i)))
    return out


# --------------------------------------------------------------------------
# the paper's evaluation circuits
# --------------------------------------------------------------------------

def qft(n: int) -> Circuit:
    """QFT staircase as drawn in the Sec. IV-A figure: for each qubit j from 0
    upward, H on j, then R_m on j controlled by qubit j+m-1 for m = 2.. .  No
    final swaps.  R_m is recorded as kind "P" with angle 2 pi / 2^m."""
    gates = []
    for j in range(n):
        gates.append(Gate("H", j))
        for m in range(2, n - j + 1):
            gates.append(Gate("P", j, (j + m - 1,), (), TWO_PI / (1 << m)))
    return Circuit(n, gates, meta={"name": "qft"})


def stream(n: int) -> Circuit:
    """Streaming circuit of the Sec. IV-C figure: gate j is X on qubit j
    controlled by qubits 0..j-1, for j = 0..n-1 in drawn order."""
    gates = [Gate("X", j, tuple(range(j))) for j in range(n)]
    return Circuit(n, gates, meta={"name": "stream"})


def ghz(n: int) -> Circuit:
    gates = [Gate("H", 0)] + [Gate("X", q + 1, (q,)) for q in range(n - 1)]
    return Circuit(n, gates, meta={"name": "ghz"})


def inverse(c: Circuit) -> Circuit:
    """Reversed gate order with each gate marked for inversion (kind prefixed
    by '~'); each side builds the adjoint matrix itself."""
    gates = [Gate("~" + g.kind, g.target, g.controls, g.values, g.theta, g.param, g.matrix)
             for g in reversed(c.gates)]
    return Circuit(c.n, gates, c.params, meta=dict(c.meta, inverse=True))
