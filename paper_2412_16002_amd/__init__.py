"""MI355X-native bound-preserving compact-stencil RKDG (cRKDG) hot path.

The compute lives in the HIP library libcrkdg.so (C ABI: include/crkdg.h);
`paper_2412_16002_amd.crkdg` is its ctypes binding and
`paper_2412_16002_amd.inputs` holds the seeded synthetic workloads.  The
binding is imported lazily so that the input generators can be used without
a GPU.

A run of the 2D Voronoi Euler workload in the mixed form (torch provides
device memory; every step runs in the library's kernels)::

    import torch
    from paper_2412_16002_amd import crkdg, inputs

    case = inputs.euler_2d_voronoi(seed=0, n=256)
    mesh = crkdg.Mesh(crkdg.problem_from_params(dict(case.params, precision="mixed")))
    slots = mesh.new_slots()                 # ring of s + 1 states
    avg, hi = mesh.views(slots[0])           # avg [V, Nc] FP64, hi [V, M-1, Nc]
    avg.copy_(torch.from_numpy(case.cell_states.T.copy()))
    hi.zero_()
    ctl = mesh.new_ctl()
    mesh.limit(slots[0], ctl)                # limited initial data
    mesh.start(slots, ctl, t_end=1e-4)       # trial dt from the wave speeds
    while mesh.ctl_read(ctl)[0]["status"] == 0:   # S_DONE at t_end
        mesh.step(slots, ctl)                # one accepted step per call
    u = slots[mesh.ctl_read(ctl)[0]["cur"]]  # the state at t_end
    print(mesh.totals(u))                    # conserved totals

Batches: pass a list of problems to `Mesh`; `mesh.autotune(slots, ctl)`
picks launch shapes and `mesh.graph(slots, ctl, attempts)` captures step
attempts in one replayable graph.
"""

__all__ = ["crkdg", "inputs", "build"]
