"""Seeded synthetic hazy inputs shared by the oracle tests, the GPU tests and the benchmark."""
from .frames import (  # noqa: F401
    A_BASE, RESOLUTIONS, Frame, Scene, StreamSpec, Video, batch_shapes_c4, haze,
    make_frame, make_scene, make_streams, make_video, quantize_u8, sha256_u8,
)
