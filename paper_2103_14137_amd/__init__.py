"""MI355X-native irradiance-matrix engine for UV coverage planning
(arXiv 2103.14137).

    paper_2103_14137_amd.uvc        binding of the HIP library (libuvc.so)
    paper_2103_14137_amd.workloads  seeded synthetic scenes, poses, lamps
    paper_2103_14137_amd.build      hipcc build of csrc/ into libuvc.so

The binding is imported lazily so that input generation needs neither torch
nor a GPU.
"""
__all__ = ["uvc", "workloads", "build"]
