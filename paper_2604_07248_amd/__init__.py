"""MI355X-native split-step turbulence propagator (TurPy hot path, arXiv 2604.07248).

    from paper_2604_07248_amd import api, workloads
    plan = api.Plan(workloads.headline().path)
    u_out = plan.propagate(u_in, seed=1)

The compute lives in libturpy.so (HIP, gfx950; C ABI in include/turpy.h);
`binding` marshals arguments, `api` adds PyTorch tensors and streams.  Submodules
load lazily so that the workload catalogue imports without the library.
"""

__all__ = ["api", "binding", "build", "workloads"]
