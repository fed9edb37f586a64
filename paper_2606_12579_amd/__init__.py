"""MI355X-native (gfx950) batched multi-agent circular-field rollout (G-MAPP hot path).

The compute lives in the HIP library libgmapp.so behind the C ABI of
include/gmapp.h; `paper_2606_12579_amd.gmapp` is its Python binding and
`paper_2606_12579_amd.scenes` the seeded synthetic input generators.
"""
__all__ = ["gmapp", "scenes"]
