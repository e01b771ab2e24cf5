"""Dense linear-algebra pins for small registers (n <= 10).

Everything here is built from Kronecker products of 2x2 matrices with numpy,
independently of the oracle's index loops: qubit q is bit q of the index, so
the full operator is kron(op_{n-1}, ..., op_1, op_0).
"""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def kron_ops(ops_by_qubit, n):
    """kron over qubits n-1 .. 0 of ops_by_qubit.get(q, I)."""
    M = np.ones((1, 1), dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        M = np.kron(M, ops_by_qubit.get(q, I2))
    return M


def controlled_unitary(n, target, controls, values, G):
    """P_sat (x) G + (I - P_sat) (x) I, P_sat = product of control projectors."""
    vals = values if len(values) else [1] * len(controls)
    proj = {q: (P1 if v else P0) for q, v in zip(controls, vals)}
    sat = kron_ops({**proj, target: np.asarray(G, dtype=np.complex128)}, n)
    sat_id = kron_ops(proj, n)
    return sat + (np.eye(1 << n, dtype=np.complex128) - sat_id)


def pauli_matrix(n, x_mask, z_mask):
    """i^{|x&z|} X^x Z^z as a dense matrix (Z applied first)."""
    ops = {}
    for q in range(n):
        xb, zb = (x_mask >> q) & 1, (z_mask >> q) & 1
        if xb and zb:
            ops[q] = PY  # i X Z = Y
        elif xb:
            ops[q] = PX
        elif zb:
            ops[q] = PZ
    return kron_ops(ops, n)


def hamiltonian_matrix(n, terms):
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for t in terms:
        H += t.coef * pauli_matrix(n, t.x_mask, t.z_mask)
    return H
