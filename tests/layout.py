"""State layout conversion between the oracle ([i][l][z][y][x]) and the library
ABI ([z][y][i][l][x]).  Both are plain array permutations."""
import numpy as np


def to_abi(y):
    return np.ascontiguousarray(np.asarray(y).transpose(2, 3, 0, 1, 4))


def from_abi(y):
    return np.ascontiguousarray(np.asarray(y).transpose(2, 3, 0, 1, 4))
