"""Loader for the small text fixtures under tests/golden/ (values printed in
the paper, each file citing where)."""
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def table(name: str) -> np.ndarray:
    """Numeric rows of a fixture (comment lines start with '#')."""
    return np.atleast_2d(np.loadtxt(os.path.join(HERE, name), comments="#"))
