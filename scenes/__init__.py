"""Seeded synthetic scenes shaped like the paper's experiments.

Every scene is built from ``numpy.random.Generator(PCG64([seed, stream]))``
and holds only inputs: meshes, the embedding matrix W (CSR), reduced
coordinates q, static/kinematic offsets, a displacement dq for the CCD bound,
and the contact parameters.  Nothing here evaluates the contact stage.
"""
from .scene import Scene, config1, tiny_scene, config3, config2, batch_scenes, full_space_scene, single_tet_scene, mixed_scale_scene  # noqa: F401
