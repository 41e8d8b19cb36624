"""Device-side helpers for the GPU tests: move seeded inputs to the device and
call the library through the C ABI (via the ctypes binding)."""
import numpy as np
import torch

from paper_1910_01260_amd import strom
from paper_1910_01260_amd import workloads as W


def colmajor(a: np.ndarray) -> torch.Tensor:
    """Device tensor with column-major storage (its transpose is contiguous)."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return torch.tensor(np.ascontiguousarray(a.T), device="cuda").T


class DeviceRom:
    """ROM buffer built on the device from given bases (st_assemble)."""

    def __init__(self, prob, Phi_s: np.ndarray, Phi_t_list, proj_prec=strom.ST_F64, integrator=strom.ST_BACKWARD_EULER):
        self.prob = prob
        n_t = [P.shape[1] for P in Phi_t_list]
        self.desc = strom.RomDesc(n_t, prob.N_t, prob.Q, prob.Qf, prob.Q0, integrator)
        self.Phi_s = colmajor(Phi_s)
        self.Phi_t = colmajor(np.concatenate(Phi_t_list, axis=1))
        self.dt = torch.tensor(prob.dt, device="cuda")
        self.csr = [strom.csr_to_device(*W.csr_arrays(A)) for A in prob.terms]
        self.Bf = colmajor(prob.Bf) if prob.Qf else None
        self.g = colmajor(prob.g) if prob.Qf else None
        self.u0 = colmajor(prob.u0) if prob.Q0 else None
        self.rom = strom.st_assemble(self.desc, self.Phi_s, self.Phi_t, self.dt, [c[0] for c in self.csr], self.Bf,
                                     self.g, self.u0, proj_prec)
        torch.cuda.synchronize()

    def section(self, name):
        return strom.rom_section(self.desc, self.rom, name)


def thetas_device(prob, mus):
    tA, tf, t0 = prob.thetas(mus)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda") if a.shape[1] else None
    return (tA, tf, t0), (dev(tA), dev(tf), dev(t0))
