"""ctypes binding of libgdm (include/gdm.h).

Argument marshalling only: every step of the density-matrix path runs in the
HIP kernels of libgdm.so.  PyTorch provides device memory and the stream.
The library must be built (``python -m paper_2606_03140_amd.build``);
importing this module without it, or without a ROCm GPU, raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgdm.so")

GDM_OK = 0
ERRORS = {-1: "E_ARG", -2: "E_CAPACITY", -3: "E_NOT_PD", -4: "E_NO_BRACKET", -5: "E_NOT_CONVERGED",
          -6: "E_NAN", -7: "E_HIP", -8: "E_STATE"}
GRAPH_CUTOFF, GRAPH_DM, GRAPH_ADAPTIVE = 0, 1, 2
FP64_EIG, MIXED_F16, MIXED_BF16 = 0, 1, 2

EXPORTED = ["gdm_create", "gdm_destroy", "gdm_set_stream", "gdm_last_error", "gdm_check", "gdm_build_graph",
            "gdm_grid_cores", "gdm_extract_subgraphs", "gdm_build_hs", "gdm_plan", "gdm_find_mu",
            "gdm_subgraph_density", "gdm_mulliken_charges", "gdm_profile", "gdm_profile_query",
            "gdm_set_mixed_options", "gdm_mixed_stats", "gdm_debug_slot"]


class GDMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class SystemT(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("pos", C.c_void_p), ("species", C.c_void_p), ("anchor", C.c_void_p),
                ("orb_ptr", C.c_void_p), ("box", C.c_double * 3), ("inv_box", C.c_double * 3)]


class TBParamsT(C.Structure):
    _fields_ = [("onsite", (C.c_double * 4) * 2), ("n_orb", C.c_int32 * 2), ("v0", C.c_double),
                ("v_r0", C.c_double), ("v_decay", C.c_double), ("s0", C.c_double), ("s_r0", C.c_double),
                ("s_decay", C.c_double), ("cutoff", C.c_double), ("orthogonal", C.c_int32),
                ("taper_on", C.c_double), ("rep_A", C.c_double * 3), ("rep_rho", C.c_double)]


class SubgraphsT(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("atom_ptr", C.c_void_p), ("atoms", C.c_void_p), ("n_core", C.c_void_p),
                ("h_norb", C.c_void_p), ("h_ncore_orb", C.c_void_p)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"libgdm is not built ({path} missing): run python -m paper_2606_03140_amd.build")
    lib = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "gdm_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, P]),
        "gdm_destroy": (C.c_int, [P]),
        "gdm_set_stream": (C.c_int, [P, P]),
        "gdm_last_error": (C.c_char_p, [P]),
        "gdm_check": (C.c_int, [P]),
        "gdm_build_graph": (C.c_int, [P, C.POINTER(SystemT), C.c_int, D, D, D, C.POINTER(SubgraphsT), P, P, P, P, P,
                                      P, P, I64, C.POINTER(C.c_int64)]),
        "gdm_grid_cores": (C.c_int, [P, C.POINTER(SystemT), C.POINTER(C.c_int32), P, C.POINTER(C.c_int32)]),
        "gdm_extract_subgraphs": (C.c_int, [P, C.POINTER(SystemT), C.POINTER(TBParamsT), P, P, P, I32, P, P, I64, P,
                                            P, P, C.POINTER(C.c_int64)]),
        "gdm_build_hs": (C.c_int, [P, C.POINTER(SystemT), C.POINTER(TBParamsT), P, P, I64, P, P, P]),
        "gdm_plan": (C.c_int, [P, C.POINTER(SubgraphsT), C.c_int]),
        "gdm_find_mu": (C.c_int, [P, C.POINTER(SystemT), C.POINTER(SubgraphsT), P, P, I64, P, P, D, D, C.c_int, D, D,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "gdm_subgraph_density": (C.c_int, [P, C.POINTER(SubgraphsT), D, D, C.c_int, P, P]),
        "gdm_mulliken_charges": (C.c_int, [P, C.POINTER(SystemT), C.POINTER(SubgraphsT), P, P, I64, P, P,
                                           C.POINTER(C.c_double), P]),
    }
    sig["gdm_set_mixed_options"] = (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int])
    sig["gdm_set_mu_outputs"] = (C.c_int, [P, C.c_int])
    sig["gdm_set_mixed_storage"] = (C.c_int, [P, C.c_int])
    sig["gdm_set_mixed_inverse_start"] = (C.c_int, [P, C.c_int])
    sig["gdm_set_mixed_capture"] = (C.c_int, [P, C.c_int, C.c_int])
    sig["gdm_mixed_mu_state"] = (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)])
    sig["gdm_subgraph_density_dmu"] = (C.c_int, [P, C.POINTER(SubgraphsT), P, D, C.c_int, P])
    sig["gdm_mixed_stats"] = (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int)])
    sig["gdm_debug_slot"] = (C.c_int, [P, C.c_int, C.c_int, P])
    sig["gdm_balanced_cores"] = (C.c_int, [P, C.POINTER(SystemT), P, I32, P])
    sig["gdm_rcb_partition"] = (C.c_int, [P, P, I32, I32, P])
    sig["gdm_set_fp64_options"] = (C.c_int, [P, C.c_int])
    sig["gdm_ewald_potential"] = (C.c_int, [P, C.POINTER(SystemT), P, P, D, D, I32, C.POINTER(C.c_double),
                                            C.POINTER(C.c_double), P, P])
    sig["gdm_ewald_potential_noalloc"] = (C.c_int, [P, C.POINTER(SystemT), P, P, D, D, I32, C.POINTER(C.c_double),
                                                    C.POINTER(C.c_double), P, P])
    sig["gdm_scc_mix"] = (C.c_int, [P, I32, P, P, D, C.POINTER(C.c_double)])
    sig["gdm_scc_anderson"] = (C.c_int, [P, I32, P, P, D, I32, I32, P, C.POINTER(C.c_double)])
    sig["gdm_set_response"] = (C.c_int, [P, C.c_int])
    sig["gdm_density_response"] = (C.c_int, [P, C.POINTER(SystemT), C.POINTER(SubgraphsT), P, P, I64, P, P, P,
                                             C.POINTER(C.c_double)])
    sig["gdm_krylov_begin"] = (C.c_int, [P, I32, P, P, D, I32, P, C.POINTER(C.c_double)])
    sig["gdm_krylov_add"] = (C.c_int, [P, I32, I32, P, I32, P, C.POINTER(C.c_double), C.POINTER(C.c_int32)])
    sig["gdm_krylov_apply"] = (C.c_int, [P, I32, I32, I32, D, I32, P, P])
    sig["gdm_descriptors"] = (C.c_int, [P, C.POINTER(SystemT), P, P, P])
    sig["gdm_feature_sums"] = (C.c_int, [P, I32, P, P, P])
    sig["gdm_feature_norm"] = (C.c_int, [P, P, P])
    sig["gdm_mlp_forward"] = (C.c_int, [P, I32, P, P, P, P, C.c_int, P])
    sig["gdm_mlp_charges"] = (C.c_int, [P, I32, P, P])
    sig["gdm_mlp_loss"] = (C.c_int, [P, I32, P, P, P])
    sig["gdm_mlp_backward"] = (C.c_int, [P, I32, P, P, P, P, P, P, P, P, P])
    sig["gdm_adam_step"] = (C.c_int, [P, I32, P, P, P, P, I32, C.c_float, C.c_float, C.c_float, C.c_float])
    sig["gdm_subgraph_edm"] = (C.c_int, [P, C.POINTER(SubgraphsT), D, D, P])
    sig["gdm_band_energy"] = (C.c_int, [P, C.POINTER(SubgraphsT), D, D, C.POINTER(C.c_double)])
    sig["gdm_forces"] = (C.c_int, [P, C.POINTER(SystemT), C.POINTER(TBParamsT), P, P, I64, C.POINTER(SubgraphsT), P,
                                   P, P, C.POINTER(C.c_double), P, P, P])
    sig["gdm_ewald_forces"] = (C.c_int, [P, C.POINTER(SystemT), P, P, D, D, I32, C.POINTER(C.c_double), P, P, P])
    sig["gdm_md_verlet"] = (C.c_int, [P, I32, P, C.POINTER(C.c_double), D, P, P, P, P])
    sig["gdm_xlbomd_charges"] = (C.c_int, [P, I32, P, P, P, D, D, P])
    sig["gdm_axpby"] = (C.c_int, [P, I32, D, P, D, P, P])
    sig["gdm_profile"] = (C.c_int, [P, C.c_int])
    sig["gdm_profile_query"] = (C.c_int, [P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)])
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def rcb_partition(xyz: np.ndarray, n_parts: int, weight: np.ndarray | None = None) -> np.ndarray:
    """Weighted recursive coordinate bisection on host arrays
    (gdm_rcb_partition; runs on the host, no GPU)."""
    x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    w = None if weight is None else np.ascontiguousarray(weight, dtype=np.float64)
    part = np.zeros(len(x), dtype=np.int32)
    rc = lib().gdm_rcb_partition(x.ctypes.data_as(C.c_void_p), None if w is None else w.ctypes.data_as(C.c_void_p),
                                 len(x), int(n_parts), part.ctypes.data_as(C.c_void_p))
    if rc:
        raise GDMError(rc, f"gdm_rcb_partition: error {rc}")
    return part


def _ptr(t):
    return C.c_void_p(0) if t is None else C.c_void_p(t.data_ptr())


@dataclass
class TBParams:
    """Synthetic two-centre model (water-like stand-in for SCC-DFTB tables)."""
    eps_s_O: float = -23.9
    eps_p_O: float = -9.0
    eps_s_H: float = -6.4
    v0: float = -4.0
    v_r0: float = 1.0
    v_decay: float = 0.5
    s0: float = 0.3
    s_r0: float = 1.0
    s_decay: float = 0.6
    cutoff: float = 4.0
    orthogonal: bool = False
    taper_on: float = 0.0              # > 0: radial functions tapered to 0 between taper_on and cutoff
    rep_A: tuple = (0.0, 0.0, 0.0)     # repulsive pair prefactors (eV): O-O, O-H, H-H
    rep_rho: float = 0.3               # repulsive decay length (A)

    def struct(self) -> TBParamsT:
        p = TBParamsT()
        for a, v in enumerate((self.eps_s_O, self.eps_p_O, self.eps_p_O, self.eps_p_O)):
            p.onsite[0][a] = v
        p.onsite[1][0] = self.eps_s_H
        p.n_orb[0], p.n_orb[1] = 4, 1
        p.v0, p.v_r0, p.v_decay = self.v0, self.v_r0, self.v_decay
        p.s0, p.s_r0, p.s_decay = self.s0, self.s_r0, self.s_decay
        p.cutoff = self.cutoff
        p.orthogonal = int(self.orthogonal)
        p.taper_on = float(self.taper_on)
        for i in range(3):
            p.rep_A[i] = float(self.rep_A[i])
        p.rep_rho = float(self.rep_rho)
        return p


N_ORB = (4, 1)
VALENCE = (6.0, 1.0)


class System:
    """Device-resident system description (positions, species, anchors, orbital offsets)."""

    def __init__(self, pos, species, anchor, box, device="cuda"):
        species = np.asarray(species, dtype=np.int32)
        self.n_atoms = int(species.shape[0])
        self.pos = torch.as_tensor(np.ascontiguousarray(pos, dtype=np.float64)).to(device)
        self.species = torch.as_tensor(species).to(device)
        self.anchor = torch.as_tensor(np.asarray(anchor, dtype=np.int32)).to(device)
        norb = np.array(N_ORB, dtype=np.int32)[species]
        orb_ptr = np.zeros(self.n_atoms + 1, dtype=np.int32)
        orb_ptr[1:] = np.cumsum(norb)
        self.n_orb = int(orb_ptr[-1])
        self.orb_ptr = torch.as_tensor(orb_ptr).to(device)
        self.box = [float(b) for b in box]
        self.inv_box = [1.0 / b for b in self.box]
        self.n_electrons = float(np.array(VALENCE)[species].sum())
        self.h_species = species

    def set_positions(self, pos):
        self.pos.copy_(torch.as_tensor(np.ascontiguousarray(pos, dtype=np.float64)))

    def struct(self) -> SystemT:
        s = SystemT()
        s.n_atoms = self.n_atoms
        s.pos, s.species, s.anchor, s.orb_ptr = (self.pos.data_ptr(), self.species.data_ptr(),
                                                 self.anchor.data_ptr(), self.orb_ptr.data_ptr())
        for a in range(3):
            s.box[a] = self.box[a]
            s.inv_box[a] = self.inv_box[a]
        return s


@dataclass
class Graph:
    row_ptr: torch.Tensor
    col: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col.numel())


class Subgraphs:
    def __init__(self, atom_ptr, atoms, n_core, norb, ncore_orb):
        self.atom_ptr, self.atoms, self.n_core = atom_ptr, atoms, n_core
        self.norb = np.ascontiguousarray(norb, dtype=np.int32)
        self.ncore_orb = np.ascontiguousarray(ncore_orb, dtype=np.int32)
        self.n_sub = int(self.norb.shape[0])
        dc = (self.norb.astype(np.int64) * self.ncore_orb)
        self.dcore_off = np.concatenate([[0], np.cumsum(dc)])
        self.eig_off = np.concatenate([[0], np.cumsum(self.norb.astype(np.int64))])

    def struct(self) -> SubgraphsT:
        s = SubgraphsT()
        s.n_sub = self.n_sub
        s.atom_ptr, s.atoms, s.n_core = self.atom_ptr.data_ptr(), self.atoms.data_ptr(), self.n_core.data_ptr()
        s.h_norb = self.norb.ctypes.data
        s.h_ncore_orb = self.ncore_orb.ctypes.data
        return s

    def host_lists(self):
        ap = self.atom_ptr.cpu().numpy()
        at = self.atoms.cpu().numpy()
        nc = self.n_core.cpu().numpy()
        return [(at[ap[s]:ap[s + 1]].astype(np.int64), int(nc[s])) for s in range(self.n_sub)]


class Context:
    """One libgdm context on a device and the current torch stream."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libgdm needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = device
        self.dev = torch.device("cuda", device)
        self.lib = lib()
        h = C.c_void_p()
        stream = torch.cuda.current_stream(self.dev).cuda_stream
        self._check(self.lib.gdm_create(C.byref(h), device, C.c_void_p(stream)), ctx=None)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.gdm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, ctx="self"):
        if rc != GDM_OK:
            msg = "" if ctx is None else self.lib.gdm_last_error(self.h).decode()
            raise GDMError(rc, msg)

    def sync_stream(self):
        self._check(self.lib.gdm_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)))

    # ---------------------------------------------------------------- graph
    def build_graph_cutoff(self, system: System, cutoff: float = 4.0) -> Graph:
        row_ptr = torch.empty(system.n_atoms + 1, dtype=torch.int32, device=self.dev)
        nnz = C.c_int64(0)
        cap = 64 * system.n_atoms
        for _ in range(2):
            col = torch.empty(max(cap, 1), dtype=torch.int32, device=self.dev)
            rc = self.lib.gdm_build_graph(self.h, C.byref(system.struct()), GRAPH_CUTOFF, cutoff, 0.0, 0.0, None, None,
                                          None, None, None, None, _ptr(row_ptr), _ptr(col), cap, C.byref(nnz))
            if rc == -2:
                cap = int(nnz.value)
                continue
            self._check(rc)
            break
        return Graph(row_ptr, col[:nnz.value])

    def build_graph_dm(self, system: System, mode: int, prev: "Subgraphs", D_core: torch.Tensor, tau: float,
                       alpha: float = 0.7, nbr: Graph | None = None, union: Graph | None = None) -> Graph:
        row_ptr = torch.empty(system.n_atoms + 1, dtype=torch.int32, device=self.dev)
        nnz = C.c_int64(0)
        cap = 128 * system.n_atoms
        for _ in range(2):
            col = torch.empty(max(cap, 1), dtype=torch.int32, device=self.dev)
            rc = self.lib.gdm_build_graph(
                self.h, C.byref(system.struct()), mode, 0.0, alpha, tau, C.byref(prev.struct()), _ptr(D_core),
                _ptr(nbr.row_ptr if nbr else None), _ptr(nbr.col if nbr else None),
                _ptr(union.row_ptr if union else None), _ptr(union.col if union else None),
                _ptr(row_ptr), _ptr(col), cap, C.byref(nnz))
            if rc == -2 and nnz.value > cap:
                cap = int(nnz.value)
                continue
            self._check(rc)
            break
        return Graph(row_ptr, col[:nnz.value])

    # ------------------------------------------------------------ partition
    def grid_cores(self, system: System, grid) -> tuple[torch.Tensor, int]:
        core = torch.empty(system.n_atoms, dtype=torch.int32, device=self.dev)
        g = (C.c_int32 * 3)(*[int(x) for x in grid])
        n = C.c_int32(0)
        self._check(self.lib.gdm_grid_cores(self.h, C.byref(system.struct()), g, _ptr(core), C.byref(n)))
        return core, int(n.value)

    def set_fp64_options(self, leaf_rows: int = 64):
        """Largest leaf of the FP64 path's divide and conquer (next plan)."""
        self._check(self.lib.gdm_set_fp64_options(self.h, int(leaf_rows)))

    def balanced_cores(self, system: System, n_cores: int, graph: Graph | None = None) -> torch.Tensor:
        """Cost-balanced cores (weighted recursive bisection; gdm_balanced_cores)."""
        core = torch.empty(system.n_atoms, dtype=torch.int32, device=self.dev)
        self._check(self.lib.gdm_balanced_cores(self.h, C.byref(system.struct()),
                                                _ptr(graph.row_ptr) if graph is not None else None, int(n_cores),
                                                _ptr(core)))
        return core

    def extract_subgraphs(self, system: System, tb: TBParams, graph: Graph, core_of_atom, n_cores) -> Subgraphs:
        atom_ptr = torch.empty(n_cores + 1, dtype=torch.int32, device=self.dev)
        n_core = torch.empty(n_cores, dtype=torch.int32, device=self.dev)
        norb = np.zeros(n_cores, dtype=np.int32)
        ncore_orb = np.zeros(n_cores, dtype=np.int32)
        total = C.c_int64(0)
        cap = 16 * system.n_atoms
        for _ in range(2):
            atoms = torch.empty(max(cap, 1), dtype=torch.int32, device=self.dev)
            rc = self.lib.gdm_extract_subgraphs(self.h, C.byref(system.struct()), C.byref(tb.struct()),
                                                _ptr(graph.row_ptr), _ptr(graph.col), _ptr(core_of_atom), n_cores,
                                                _ptr(atom_ptr), _ptr(atoms), cap, _ptr(n_core),
                                                C.c_void_p(norb.ctypes.data), C.c_void_p(ncore_orb.ctypes.data),
                                                C.byref(total))
            if rc == -2 and total.value > cap:
                cap = int(total.value)
                continue
            self._check(rc)
            break
        return Subgraphs(atom_ptr, atoms[:total.value], n_core, norb, ncore_orb)

    # --------------------------------------------------------------- H and S
    def build_hs(self, system: System, tb: TBParams, graph: Graph, V_atom: torch.Tensor | None = None):
        nb = (graph.nnz + system.n_atoms) * 16
        H = torch.empty(nb, dtype=torch.float64, device=self.dev)
        S = None if tb.orthogonal else torch.empty(nb, dtype=torch.float64, device=self.dev)
        self._check(self.lib.gdm_build_hs(self.h, C.byref(system.struct()), C.byref(tb.struct()), _ptr(graph.row_ptr),
                                          _ptr(graph.col), graph.nnz, _ptr(V_atom), _ptr(H), _ptr(S)))
        return H, S

    # ----------------------------------------------------------------- solve
    def plan(self, sg: Subgraphs, precision: int):
        self._check(self.lib.gdm_plan(self.h, C.byref(sg.struct()), precision))

    def find_mu(self, system: System, sg: Subgraphs, graph: Graph, H, S, kT: float, precision: int,
                mu_guess: float = 0.0, tol_N: float = 1e-6, n_electrons: float | None = None):
        mu = C.c_double(0.0)
        n = C.c_double(0.0)
        ne = system.n_electrons if n_electrons is None else n_electrons
        self._check(self.lib.gdm_find_mu(self.h, C.byref(system.struct()), C.byref(sg.struct()), _ptr(graph.row_ptr),
                                         _ptr(graph.col), graph.nnz, _ptr(H), _ptr(S), ne, kT, precision, mu_guess,
                                         tol_N, C.byref(mu), C.byref(n)))
        return mu.value, n.value

    def set_mu_outputs(self, device: bool):
        """device=True: find_mu_device writes mu and N(mu) to device scalars
        without synchronising (both paths; the mixed path then searches with a
        fixed number of predicated passes, set_mixed_capture)."""
        self._check(self.lib.gdm_set_mu_outputs(self.h, 1 if device else 0))

    def set_mixed_capture(self, passes: int, nd_launch: int):
        self._check(self.lib.gdm_set_mixed_capture(self.h, int(passes), int(nd_launch)))

    def mixed_mu_state(self) -> dict:
        mp, npass, sl = C.c_double(0.0), C.c_double(0.0), C.c_double(0.0)
        self._check(self.lib.gdm_mixed_mu_state(self.h, C.byref(mp), C.byref(npass), C.byref(sl)))
        return {"mu_pass": mp.value, "n_pass": npass.value, "slope": sl.value}

    def find_mu_device(self, system: System, sg: Subgraphs, graph: Graph, H, S, kT: float, precision: int,
                       mu_out: torch.Tensor, n_out: torch.Tensor, n_electrons: float | None = None,
                       mu_guess: float = 0.0, tol_N: float = 0.0):
        """gdm_find_mu with DEVICE outputs (after set_mu_outputs(True)): mu_out and
        n_out are float64 device tensors of one element, written on the stream
        (the mixed path starts from mu_out's value when it is finite and inside
        the spectral bounds, else from mu_guess)."""
        ne = system.n_electrons if n_electrons is None else n_electrons
        self._check(self.lib.gdm_find_mu(self.h, C.byref(system.struct()), C.byref(sg.struct()), _ptr(graph.row_ptr),
                                         _ptr(graph.col), graph.nnz, _ptr(H), _ptr(S), ne, kT, precision, mu_guess,
                                         tol_N, C.cast(_ptr(mu_out), C.POINTER(C.c_double)),
                                         C.cast(_ptr(n_out), C.POINTER(C.c_double))))

    def subgraph_density_dmu(self, sg: Subgraphs, mu_device: torch.Tensor, kT: float, precision: int,
                             out: torch.Tensor):
        """D core rows at the chemical potential held in the device scalar mu_device."""
        self._check(self.lib.gdm_subgraph_density_dmu(self.h, C.byref(sg.struct()), _ptr(mu_device), kT, precision,
                                                      _ptr(out)))
        return out

    def subgraph_density(self, sg: Subgraphs, mu: float, kT: float, precision: int, eig: bool = False,
                         out: torch.Tensor | None = None):
        D = out if out is not None else torch.empty(int(sg.dcore_off[-1]), dtype=torch.float64, device=self.dev)
        E = torch.empty(int(sg.eig_off[-1]), dtype=torch.float64, device=self.dev) if eig else None
        self._check(self.lib.gdm_subgraph_density(self.h, C.byref(sg.struct()), mu, kT, precision, _ptr(D), _ptr(E)))
        return (D, E) if eig else D

    def mulliken_charges(self, system: System, sg: Subgraphs, graph: Graph, S, D_core, out=None):
        q = out if out is not None else torch.empty(system.n_atoms, dtype=torch.float64, device=self.dev)
        n0 = (C.c_double * 2)(*VALENCE)
        self._check(self.lib.gdm_mulliken_charges(self.h, C.byref(system.struct()), C.byref(sg.struct()),
                                                  _ptr(graph.row_ptr), _ptr(graph.col), graph.nnz, _ptr(S),
                                                  _ptr(D_core), n0, _ptr(q)))
        return q

    # ------------------------------------------------------ forces (XL-BOMD)
    def subgraph_edm(self, sg: Subgraphs, mu: float, kT: float, out: torch.Tensor | None = None):
        """Energy-weighted density core rows (FP64 path, after find_mu)."""
        W = out if out is not None else torch.empty(int(sg.dcore_off[-1]), dtype=torch.float64, device=self.dev)
        self._check(self.lib.gdm_subgraph_edm(self.h, C.byref(sg.struct()), mu, kT, _ptr(W)))
        return W

    def band_energy(self, sg: Subgraphs, mu: float, kT: float) -> float:
        e = C.c_double(0.0)
        self._check(self.lib.gdm_band_energy(self.h, C.byref(sg.struct()), mu, kT, C.byref(e)))
        return e.value

    def forces(self, system: System, tb: TBParams, graph: Graph, sg: Subgraphs, D_core, W_core, V_atom=None,
               n_vec=None, out: torch.Tensor | None = None, energy: torch.Tensor | None = None):
        """Band, Pulay, SCC-shift and repulsive forces [n_atoms, 3]; energy
        (device [2], optional): repulsion and -sum (n0 + n/2) V."""
        F = out if out is not None else torch.empty(system.n_atoms, 3, dtype=torch.float64, device=self.dev)
        n0 = (C.c_double * 2)(*VALENCE)
        self._check(self.lib.gdm_forces(self.h, C.byref(system.struct()), C.byref(tb.struct()), _ptr(graph.row_ptr),
                                        _ptr(graph.col), graph.nnz, C.byref(sg.struct()), _ptr(D_core),
                                        _ptr(W_core), _ptr(V_atom), n0, _ptr(n_vec), _ptr(F), _ptr(energy)))
        return F

    def ewald_forces(self, system: System, graph: Graph, rcut: float, eta: float, k_max: int, q, n_vec, F,
                     tau=None):
        """F += -d/dR (1/2 (2q - n)^T gamma n) (Coulomb part of the shadow forces)."""
        T = None if tau is None else (C.c_double * 2)(*[float(t) for t in tau])
        self._check(self.lib.gdm_ewald_forces(self.h, C.byref(system.struct()), _ptr(graph.row_ptr),
                                              _ptr(graph.col), rcut, eta, int(k_max), T, _ptr(q), _ptr(n_vec),
                                              _ptr(F)))
        return F

    def md_verlet(self, system: System, mass, dt: float, F, vel, drift: bool, kinetic=None):
        m = (C.c_double * 2)(*[float(x) for x in mass])
        self._check(self.lib.gdm_md_verlet(self.h, system.n_atoms, _ptr(system.species), m, dt, _ptr(F), _ptr(vel),
                                           _ptr(system.pos) if drift else C.c_void_p(0), _ptr(kinetic)))

    def xlbomd_charges(self, q, hist, kappa_c: float, alpha: float, out=None, delta=None):
        self._check(self.lib.gdm_xlbomd_charges(self.h, int(hist.shape[1]), _ptr(q), _ptr(delta), _ptr(hist),
                                                kappa_c, alpha, _ptr(out)))
        return out

    def axpby(self, a: float, x, b: float, y, out):
        """out = a x + b y (device vectors)."""
        self._check(self.lib.gdm_axpby(self.h, int(x.numel()), a, _ptr(x), b, _ptr(y), _ptr(out)))
        return out

    def check(self):
        self._check(self.lib.gdm_check(self.h))

    def set_mixed_storage(self, upper_tiles: bool):
        self._check(self.lib.gdm_set_mixed_storage(self.h, 1 if upper_tiles else 0))

    def set_mixed_inverse_start(self, degree: int):
        self._check(self.lib.gdm_set_mixed_inverse_start(self.h, int(degree)))

    def set_mixed_options(self, ns_z: int = 0, ns_inv: int = 0, max_passes: int = 0, ns_z_extra: int = -1):
        self._check(self.lib.gdm_set_mixed_options(self.h, ns_z, ns_inv, max_passes, ns_z_extra))

    def debug_slot(self, which: int, sub: int, P: int) -> torch.Tensor:
        out = torch.empty(P * P, dtype=torch.float32, device=self.dev)
        self._check(self.lib.gdm_debug_slot(self.h, which, sub, _ptr(out)))
        return out.view(P, P)

    def mixed_stats(self) -> dict:
        p, nd, g, f, b, z = C.c_int(0), C.c_int(0), C.c_int64(0), C.c_double(0.0), C.c_double(0.0), C.c_int(0)
        self._check(self.lib.gdm_mixed_stats(self.h, C.byref(p), C.byref(nd), C.byref(g), C.byref(f), C.byref(b),
                                             C.byref(z)))
        return {"passes": p.value, "n_doublings": nd.value, "gemm_launches": g.value,
                "flops_per_launch": f.value, "bytes_per_launch": b.value, "ns_z_used": z.value}

    # ------------------------------------------------------------ SCC shell
    def ewald_potential(self, system: System, graph: Graph, rcut: float, eta: float, k_max: int, hubbard_U, q,
                        tau=None, out=None):
        V = out if out is not None else torch.empty(system.n_atoms, dtype=torch.float64, device=self.dev)
        U = (C.c_double * 2)(*[float(u) for u in hubbard_U])
        T = None if tau is None else (C.c_double * 2)(*[float(t) for t in tau])
        self._check(self.lib.gdm_ewald_potential(self.h, C.byref(system.struct()), _ptr(graph.row_ptr),
                                                 _ptr(graph.col), rcut, eta, int(k_max), U, T, _ptr(q), _ptr(V)))
        return V

    def ewald_potential_noalloc(self, system: System, graph: Graph, rcut: float, eta: float, k_max: int, hubbard_U,
                               q, tau=None, out=None):
        V = out if out is not None else torch.empty(system.n_atoms, dtype=torch.float64, device=self.dev)
        U = (C.c_double * 2)(*[float(u) for u in hubbard_U])
        T = None if tau is None else (C.c_double * 2)(*[float(t) for t in tau])
        self._check(self.lib.gdm_ewald_potential_noalloc(self.h, C.byref(system.struct()), _ptr(graph.row_ptr),
                                                         _ptr(graph.col), rcut, eta, int(k_max), U, T, _ptr(q),
                                                         _ptr(V)))
        return V

    def scc_mix(self, n_vec, q0, mix: float) -> float:
        rms = C.c_double(0.0)
        self._check(self.lib.gdm_scc_mix(self.h, int(n_vec.numel()), _ptr(n_vec), _ptr(q0), mix, C.byref(rms)))
        return rms.value

    def scc_anderson(self, n_vec, q0, mix: float, depth: int, k: int, work) -> float:
        rms = C.c_double(0.0)
        self._check(self.lib.gdm_scc_anderson(self.h, int(n_vec.numel()), _ptr(n_vec), _ptr(q0), mix, int(depth),
                                              int(k), _ptr(work), C.byref(rms)))
        return rms.value

    # ---------------------------------------- response and quasi-Newton SCF
    def set_response(self, max_doublings: int):
        self._check(self.lib.gdm_set_response(self.h, int(max_doublings)))

    def density_response(self, system: System, sg: Subgraphs, graph: Graph, S, dV, out=None):
        """(dq, dmu): canonical charge response to potential change dV."""
        dq = out if out is not None else torch.empty(system.n_atoms, dtype=torch.float64, device=self.dev)
        dmu = C.c_double(0.0)
        self._check(self.lib.gdm_density_response(self.h, C.byref(system.struct()), C.byref(sg.struct()),
                                                  _ptr(graph.row_ptr), _ptr(graph.col), graph.nnz, _ptr(S),
                                                  _ptr(dV), _ptr(dq), C.byref(dmu)))
        return dq, dmu.value

    @staticmethod
    def krylov_work_size(n: int, max_rank: int) -> int:
        return (2 * max_rank + 1) * n + max_rank * max_rank + 2 * max_rank + 2

    @staticmethod
    def krylov_vector(work, n: int, j: int):
        return work[n + j * n: n + (j + 1) * n]

    def krylov_begin(self, n_vec, q0, max_rank: int, work, k0: float = 1.0) -> float:
        rms = C.c_double(0.0)
        self._check(self.lib.gdm_krylov_begin(self.h, int(n_vec.numel()), _ptr(n_vec), _ptr(q0), float(k0),
                                              int(max_rank), _ptr(work), C.byref(rms)))
        return rms.value

    def krylov_add(self, n: int, j: int, dq, max_rank: int, work) -> tuple[float, bool]:
        rel, ex = C.c_double(0.0), C.c_int32(0)
        self._check(self.lib.gdm_krylov_add(self.h, int(n), int(j), _ptr(dq), int(max_rank), _ptr(work),
                                            C.byref(rel), C.byref(ex)))
        return rel.value, bool(ex.value)

    def krylov_apply(self, n_vec, rank: int, max_rank: int, work, alpha: float = 1.0, complete: bool = False):
        self._check(self.lib.gdm_krylov_apply(self.h, int(n_vec.numel()), int(rank), int(max_rank), float(alpha),
                                              int(bool(complete)), _ptr(n_vec), _ptr(work)))

    # ------------------------------------------------------ learned guess
    def descriptors(self, system: System, graph: Graph, out=None):
        F = out if out is not None else torch.empty(system.n_atoms, 32, dtype=torch.float64, device=self.dev)
        self._check(self.lib.gdm_descriptors(self.h, C.byref(system.struct()), _ptr(graph.row_ptr), _ptr(graph.col),
                                             _ptr(F)))
        return F

    def feature_sums(self, feats, species, stats):
        self._check(self.lib.gdm_feature_sums(self.h, int(feats.shape[0]), _ptr(feats), _ptr(species), _ptr(stats)))

    def feature_norm(self, stats, norm):
        self._check(self.lib.gdm_feature_norm(self.h, _ptr(stats), _ptr(norm)))

    def mlp_forward(self, species, feats, params, norm, bf16: bool, y):
        self._check(self.lib.gdm_mlp_forward(self.h, int(species.numel()), _ptr(species), _ptr(feats), _ptr(params),
                                             _ptr(norm), int(bf16), _ptr(y)))

    def mlp_charges(self, y, q):
        self._check(self.lib.gdm_mlp_charges(self.h, int(y.numel()), _ptr(y), _ptr(q)))

    def mlp_loss(self, y, q_ref, stats3):
        self._check(self.lib.gdm_mlp_loss(self.h, int(y.numel()), _ptr(y), _ptr(q_ref), _ptr(stats3)))

    def mlp_backward(self, species, feats, params, norm, y, q_ref, stats3, partial, grad):
        self._check(self.lib.gdm_mlp_backward(self.h, int(species.numel()), _ptr(species), _ptr(feats),
                                              _ptr(params), _ptr(norm), _ptr(y), _ptr(q_ref), _ptr(stats3),
                                              _ptr(partial), _ptr(grad)))

    def adam_step(self, params, grad, m, v, t: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
                  eps: float = 1e-8):
        self._check(self.lib.gdm_adam_step(self.h, int(params.numel()), _ptr(params), _ptr(grad), _ptr(m), _ptr(v),
                                           int(t), lr, b1, b2, eps))

    # --------------------------------------------------------------- tracing
    def profile(self, enable: bool):
        self._check(self.lib.gdm_profile(self.h, int(enable)))

    def profile_query(self, kernel: str):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(self.lib.gdm_profile_query(self.h, kernel.encode(), C.byref(ms), C.byref(n)))
        return ms.value, int(n.value)
