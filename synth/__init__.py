"""Seeded synthetic bundle-adjustment workloads.

This module simulates a pinhole camera moving through a scene and records
noisy image observations of 3-D points. It is the one input source shared by
the FP64 oracle and the HIP path; it contains none of the belief-propagation
arithmetic (no linearisation, no messages, no beliefs). Rotations are built
with scipy's rotation routines so that the camera simulation shares no code
with either implementation under test.
"""
from .ba import (BAProblem, reinit_at_depth, make_config0, make_config1, make_config2,
                 make_config3_problem, make_config3, make_random_walk,
                 make_tree_chain, make_star, concat_problems, Camera,
                 IncrementalStream, make_incremental_stream)

__all__ = ["BAProblem", "reinit_at_depth", "Camera", "make_config0", "make_config1",
           "make_config2", "make_config3_problem", "make_config3",
           "make_random_walk", "make_tree_chain", "make_star",
           "concat_problems", "IncrementalStream", "make_incremental_stream"]
