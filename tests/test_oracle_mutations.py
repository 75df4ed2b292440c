"""The oracle's pins must catch plausible mistakes: each case rebuilds the
oracle on the CPU with one deliberate error (ORC_PLANT = k in oracle.cpp)
and runs every pin against it; at least one pin has to fail."""
import concurrent.futures as cf
import inspect
import os

import pytest

import oracle
import tests.test_oracle_pins as pins

PLANTS = {
    1: "compositing weight without the transmittance factor",
    2: "transmittance includes the current sample (off by one)",
    3: "encoding: cosine where the sine belongs",
    4: "encoding: frequency 2^(l+1) instead of 2^l",
    5: "MLP: square weight matrices used transposed",
    6: "MLP: ReLU of the second hidden layer dropped",
    7: "MLP: density activation ReLU instead of softplus",
    8: "traversal: sample at the segment exit instead of its midpoint",
    9: "traversal: far clip ignored",
    10: "compositing backward: wrong sign of the remaining-colour term",
    11: "equirect rays: latitude sign flipped",
    12: "global field: encoding missing from the fifth-layer input",
    13: "occupancy: logit sum not clamped to the paper's range",
    14: "occupancy: free space runs up to the depth, ignoring the uncertainty band",
    15: "occupancy: a free pass overrides a hit in the same pose",
    16: "depth statistics: weights not normalised by the opacity",
    17: "occupancy: hit logit not weakened by the uncertainty",
    18: "assignment: anchor at the largest free index",
    19: "assignment: nearest by grid steps instead of Euclidean distance",
    20: "assignment: the remainder voxels all go to the last field",
    21: "distillation: each field's term averaged over all points instead of its own",
    22: "distillation: density term left out of the gradient",
    23: "samples per voxel: pieces sampled at their start instead of their middle",
    24: "stereo rays: eye offset along the heading instead of across it",
    25: "per-field frames ignored: every field encoded in the scene frame",
    26: "local field: ReLU on the linear feature layer (forward and backward)",
    27: "global field: feature layer without its ReLU (forward and backward)",
    28: "global field: colour layer 10 without its ReLU (forward and backward)",
    29: "global field: direction encoding left out of layer 10's input",
}


def _pin_functions():
    return [(n, f) for n, f in inspect.getmembers(pins, inspect.isfunction)
            if n.startswith("test_") and list(inspect.signature(f).parameters) == ["orc"]]


@pytest.fixture(scope="module")
def mutants(tmp_path_factory):
    d = tmp_path_factory.mktemp("mutants")
    with cf.ThreadPoolExecutor(max_workers=min(8, len(PLANTS))) as ex:
        paths = dict(zip(PLANTS, ex.map(lambda k: oracle.build(out=str(d / f"liboracle_{k}.so"), plant=k), PLANTS)))
    yield paths
    oracle.use_library(None)


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_pins_catch_planted_mistake(mutants, plant):
    oracle.use_library(mutants[plant])
    failed = []
    try:
        for name, fn in _pin_functions():
            try:
                fn(oracle)
            except Exception:
                failed.append(name)
    finally:
        oracle.use_library(None)
    assert failed, f"no pin caught: {PLANTS[plant]}"


def test_unmutated_oracle_passes_every_pin():
    oracle.use_library(None)
    for name, fn in _pin_functions():
        fn(oracle)
