"""MI355X-native MPCD step with rigid-body discrete-particle colloids.

The step (site thermalization, grid shift and counting-sort binning, SRD
collision with cell thermostat, momentum transfer to the bodies, quaternion
rigid-body integration, ballistic streaming) runs as hand-written HIP kernels
for gfx950 in ``libmpcd.so``; :mod:`paper_2604_14307_amd.lib` binds its C ABI.
The library is loaded lazily so that :mod:`paper_2604_14307_amd.workloads`
can be used without a GPU.
"""

__all__ = ["lib", "workloads", "sim"]
