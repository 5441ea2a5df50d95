"""Host FP64 application of Pauli rotations to a sparse set of amplitudes
(test infrastructure for checks at sizes where no full-state oracle fits).

A rotation changes an amplitude from itself and its partner only, so after K
rotations with flip masks x_1..x_K an amplitude depends on at most 2^K
amplitudes before them: its closure under XOR with the flip masks."""
import numpy as np

from oracle import pauli


def closure(m, xs):
    out = {int(m)}
    for x in xs:
        out |= {v ^ int(x) for v in out}
    return out


def rotate_sparse(amp: dict, x, z, phi):
    """R(P, phi) = cos(phi/2) - i sin(phi/2) P on a dict of amplitudes closed
    under XOR with x (the oracle's convention: P|k> = i^{|x & z|}
    (-1)^{|k & z|} |k ^ x>)."""
    x, z = int(x), int(z)
    w = 1j ** (pauli.popcount(x & z) % 4)
    c, s = np.cos(phi / 2), np.sin(phi / 2)
    return {j: c * v - 1j * s * w * (-1) ** pauli.popcount((j ^ x) & z) * amp[j ^ x] for j, v in amp.items()}
