"""ctypes binding of libucc.so (include/ucc.h).

Argument marshalling only: every step of the computation runs in the HIP library.  With
torch CUDA tensors the device pointers and torch's current stream are passed through; with
numpy arrays the library copies to and from the host itself.  There is no CPU fallback:
if libucc.so is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libucc.so")

_i32, _u32, _u64, _dbl, _vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
_P = ctypes.POINTER

STATUS = {0: "UCC_OK", -1: "UCC_EINVAL", -2: "UCC_ENOMEM", -3: "UCC_EDEVICE", -4: "UCC_EBUSY",
          -5: "UCC_ECANCELED", -6: "UCC_ENOTFOUND"}
STATUS_CODES = {v: k for k, v in STATUS.items()}

EXPORTED = [
    "ucc_default_options", "ucc_build", "ucc_energy", "ucc_energy_grad", "ucc_energy_grad_noalloc",
    "ucc_energy_grad_jobs", "ucc_graph_status",
    "ucc_stream_probe",
    "ucc_energy_trotter_free", "ucc_energy_grad_trotter_free", "ucc_get_generator_passes",
    "ucc_get_partials_passes",
    "ucc_fmo2_energy", "ucc_get_state",
    "ucc_destroy", "ucc_last_error", "ucc_get_plan_info", "ucc_batch_compatible",
    "ucc_get_pauli_terms",
    "ucc_get_group_table", "ucc_get_excitation_table", "ucc_get_pass_table",
    "ucc_profile", "ucc_profile_read",
    "ucc_server_create", "ucc_submit", "ucc_poll", "ucc_wait", "ucc_cancel", "ucc_server_destroy",
]

KERNEL_KINDS = ["trig", "fwd", "exp", "applyh", "rev", "reduce", "whole", "gen", "cheb", "graph"]
N_KERNEL_KINDS = 10


class Options(ctypes.Structure):
    _fields_ = [("trotter_steps", _i32), ("tile_qubits", _i32), ("tile_qubits_rev", _i32),
                ("contiguous_qubits", _i32), ("block_threads", _i32), ("max_batch", _i32),
                ("launch_mode", _i32), ("host_only", _i32), ("device", _i32),
                ("block_threads_fwd", _i32), ("block_threads_exp", _i32),
                ("block_threads_rev", _i32), ("tile_qubits_exp", _i32), ("autotune", _i32),
                ("store_states", _i32), ("trotter_order", _i32), ("taper", _i32),
                ("fuse_depth", _i32), ("graph_wait_us", _i32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_qubits", _i32), ("n_elec", _i32), ("n_exc", _i32), ("n_pauli", _i32),
                ("n_groups", _i32), ("n_fwd_passes", _i32), ("n_exp_passes", _i32),
                ("n_rev_passes", _i32), ("tile_qubits", _i32), ("tile_qubits_exp", _i32),
                ("tile_qubits_rev", _i32),
                ("contiguous_fwd", _i32), ("contiguous_exp", _i32), ("contiguous_rev", _i32),
                ("block_threads_fwd", _i32), ("block_threads_exp", _i32),
                ("block_threads_rev", _i32), ("launch_mode", _i32), ("autotuned", _i32),
                ("store_states", _i32), ("trotter_steps", _i32), ("trotter_order", _i32),
                ("perm", _i32 * 32), ("job_footprint", ctypes.c_int64),
                ("state_qubits", _i32), ("taper", _i32), ("fuse_depth", _i32),
                ("graph_grid", _i32), ("graph_lds", _i32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", _i32), ("reserved", _i32), ("ms", _dbl), ("bytes", _dbl)]


class UCCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2402_17993_amd.build` (or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "ucc_default_options": (None, [_P(Options)]),
        "ucc_build": (_i32, [_i32, _i32, _vp, _vp, _vp, _i32, _P(Options), _P(_vp)]),
        "ucc_energy": (_i32, [_vp, _vp, _i32, _vp, _vp]),
        "ucc_energy_grad": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp]),
        "ucc_energy_grad_noalloc": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp]),
        "ucc_energy_grad_jobs": (_i32, [_P(_vp), _P(_i32), _P(_vp), _P(_vp), _P(_vp), _i32, _vp]),
        "ucc_graph_status": (_i32, [_vp, _vp]),
        "ucc_stream_probe": (_i32, [_vp, _vp, ctypes.c_size_t, _i32, _vp]),
        "ucc_energy_trotter_free": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp]),
        "ucc_energy_grad_trotter_free": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp, _vp]),
        "ucc_get_generator_passes": (_i32, [_vp, _i32, _vp, _vp, _P(_i32)]),
        "ucc_get_partials_passes": (_i32, [_vp, _i32, _vp, _vp, _P(_i32)]),
        "ucc_fmo2_energy": (_i32, [_i32, _vp, _vp, _P(_dbl)]),
        "ucc_get_state": (_i32, [_vp, _i32, _vp]),
        "ucc_destroy": (None, [_vp]),
        "ucc_last_error": (ctypes.c_char_p, []),
        "ucc_get_plan_info": (_i32, [_vp, _P(PlanInfo)]),
        "ucc_batch_compatible": (_i32, [_vp, _vp, _P(_i32)]),
        "ucc_get_pauli_terms": (_i32, [_vp, _vp, _vp, _vp]),
        "ucc_get_group_table": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "ucc_get_excitation_table": (_i32, [_vp, _vp, _vp, _vp, _vp]),
        "ucc_get_pass_table": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "ucc_profile": (_i32, [_vp, _i32]),
        "ucc_profile_read": (_i32, [_vp, _P(KernelStat), _i32]),
        "ucc_server_create": (_i32, [ctypes.c_size_t, _i32, _i32, _P(_vp)]),
        "ucc_submit": (_i32, [_vp, _vp, _vp, _i32, _dbl, _u32, _P(_u64)]),
        "ucc_poll": (_i32, [_vp, _u64, _P(_i32), _vp, _vp, _vp]),
        "ucc_wait": (_i32, [_vp, _u64, _vp, _vp, _vp]),
        "ucc_cancel": (_i32, [_vp, _u64]),
        "ucc_server_destroy": (None, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status, what=""):
    if status != 0:
        msg = lib().ucc_last_error().decode(errors="replace")
        raise UCCError(status, f"{what}: {msg}" if what else msg)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _torch_ready():
    try:
        import torch
    except ImportError:
        return False
    return torch.cuda.is_available() and torch.cuda.is_initialized()


def energy_grad_jobs(contexts, thetas, stream=None):
    """ucc_energy_grad_jobs: (E, dE/dtheta) of each context at its theta ([K] or [B, K]), all
    jobs in one evaluation-graph launch (contexts built with launch_mode=3).  numpy in ->
    numpy out; torch CUDA in -> torch CUDA out (every theta of one kind)."""
    L = lib()
    n = len(contexts)
    if n != len(thetas) or not 1 <= n <= 4:
        raise ValueError("one theta per context, 1 to 4 jobs")
    cuda = [_is_torch_cuda(t) for t in thetas]
    if any(cuda) and not all(cuda):
        raise ValueError("thetas must be all numpy or all torch CUDA tensors")
    keep, th_p, e_p, g_p, Bs, outs = [], [], [], [], [], []
    if all(cuda):
        import torch
        for c, t in zip(contexts, thetas):
            th = t.detach().to(torch.float64).contiguous()
            B = th.numel() // c.n_exc
            if th.numel() != B * c.n_exc or B < 1:
                raise ValueError("theta must hold B * n_exc amplitudes")
            E = torch.empty(B, dtype=torch.float64, device=th.device)
            G = torch.empty(B, c.n_exc, dtype=torch.float64, device=th.device)
            keep += [th]
            th_p.append(th.data_ptr()), e_p.append(E.data_ptr()), g_p.append(G.data_ptr())
            Bs.append(B), outs.append((E, G))
        st = stream if stream is not None else torch.cuda.current_stream(thetas[0].device).cuda_stream
    else:
        for c, t in zip(contexts, thetas):
            th = np.ascontiguousarray(t, dtype=np.float64)
            B = th.size // c.n_exc
            if th.size != B * c.n_exc or B < 1:
                raise ValueError("theta must hold B * n_exc amplitudes")
            E = np.empty(B)
            G = np.empty((B, c.n_exc))
            keep += [th, E, G]
            th_p.append(th.ctypes.data), e_p.append(E.ctypes.data), g_p.append(G.ctypes.data)
            Bs.append(B), outs.append((E, G))
        st = stream
    arr = lambda xs: (_vp * n)(*[_vp(x) for x in xs])
    check(L.ucc_energy_grad_jobs((_vp * n)(*[c._h for c in contexts]), (_i32 * n)(*Bs), arr(th_p),
                                 arr(e_p), arr(g_p), n, _vp(st) if st is not None else None),
          "ucc_energy_grad_jobs")
    return outs


def _is_torch_cuda(x):
    try:
        import torch
    except ImportError:
        return False
    return isinstance(x, torch.Tensor) and x.is_cuda


class Context:
    """One Hamiltonian (Eq. 2) + excitation list (Eqs. 4-5) + device buffers."""

    def __init__(self, n_qubits, n_elec, h1, h2, exc, *, tile_qubits=0, tile_qubits_exp=0,
                 tile_qubits_rev=0,
                 contiguous_qubits=0, block_threads=0, block_threads_fwd=0,
                 block_threads_exp=0, block_threads_rev=0, max_batch=1, launch_mode=0,
                 autotune=False, store_states=0, trotter_steps=1, trotter_order=1,
                 taper=0, fuse_depth=0, graph_wait_us=0, host_only=False, device=-1):
        L = lib()
        self._h = None
        self.n_qubits, self.n_elec = int(n_qubits), int(n_elec)
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        h2 = np.ascontiguousarray(h2, dtype=np.float64)
        exc = np.ascontiguousarray(exc, dtype=np.int32).reshape(-1, 4)
        self.n_exc = exc.shape[0]
        o = Options()
        L.ucc_default_options(ctypes.byref(o))
        o.tile_qubits, o.tile_qubits_rev = tile_qubits, tile_qubits_rev
        o.tile_qubits_exp = tile_qubits_exp
        o.contiguous_qubits, o.block_threads = contiguous_qubits, block_threads
        o.block_threads_fwd, o.block_threads_exp = block_threads_fwd, block_threads_exp
        o.block_threads_rev, o.autotune = block_threads_rev, int(bool(autotune))
        o.max_batch, o.launch_mode = max_batch, launch_mode
        o.store_states = store_states
        o.trotter_steps, o.trotter_order = trotter_steps, trotter_order
        o.taper = int(taper)
        o.fuse_depth = int(fuse_depth)
        o.graph_wait_us = int(graph_wait_us)
        o.host_only, o.device = int(bool(host_only)), device
        h = _vp()
        check(L.ucc_build(self.n_qubits, self.n_elec, _ptr(h1), _ptr(h2), _ptr(exc),
                          self.n_exc, ctypes.byref(o), ctypes.byref(h)), "ucc_build")
        self._h = h

    # ------------------------------------------------------------ evaluation
    def _run(self, theta, grad, stream):
        L = lib()
        if _is_torch_cuda(theta):
            import torch
            th = theta.detach().to(torch.float64).contiguous()
            B = th.numel() // self.n_exc
            if th.numel() != B * self.n_exc or B < 1:
                raise ValueError("theta must hold B * n_exc amplitudes")
            E = torch.empty(B, dtype=torch.float64, device=th.device)
            G = torch.empty(B, self.n_exc, dtype=torch.float64, device=th.device) if grad else None
            st = stream if stream is not None else torch.cuda.current_stream(th.device).cuda_stream
            if grad:
                check(L.ucc_energy_grad(self._h, _vp(th.data_ptr()), B, _vp(E.data_ptr()),
                                        _vp(G.data_ptr()), _vp(st)), "ucc_energy_grad")
            else:
                check(L.ucc_energy(self._h, _vp(th.data_ptr()), B, _vp(E.data_ptr()), _vp(st)),
                      "ucc_energy")
            return E, G
        th = np.ascontiguousarray(theta, dtype=np.float64)
        B = th.size // self.n_exc
        if th.size != B * self.n_exc or B < 1:
            raise ValueError("theta must hold B * n_exc amplitudes")
        E = np.empty(B)
        G = np.empty((B, self.n_exc)) if grad else None
        st = _vp(stream) if stream is not None else None
        if grad:
            check(L.ucc_energy_grad(self._h, _ptr(th), B, _ptr(E), _ptr(G), st), "ucc_energy_grad")
        else:
            check(L.ucc_energy(self._h, _ptr(th), B, _ptr(E), st), "ucc_energy")
        return E, G

    def energy(self, theta, stream=None):
        """E for theta [K] or [B, K] (numpy -> numpy, torch CUDA -> torch CUDA)."""
        return self._run(theta, False, stream)[0]

    def energy_grad(self, theta, stream=None):
        """(E [B], dE/dtheta [B, K])."""
        return self._run(theta, True, stream)

    def graph_status(self, stream=None):
        """ucc_graph_status: raises UCCError (UCC_EDEVICE) if an evaluation-graph launch of this
        context gave up waiting since the last check; synchronizes the stream first."""
        if stream is None and _torch_ready():
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        check(lib().ucc_graph_status(self._h, _vp(stream) if stream is not None else None),
              "ucc_graph_status")

    def energy_grad_noalloc(self, theta, energy, grad, stream=None):
        """ucc_energy_grad_noalloc: theta [B, K] in, energy [B] and grad [B, K] out, all
        contiguous float64 torch CUDA tensors the caller owns; the call allocates nothing."""
        import torch
        for name, t in (("theta", theta), ("energy", energy), ("grad", grad)):
            if not (_is_torch_cuda(t) and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
        B = theta.numel() // self.n_exc
        if theta.numel() != B * self.n_exc or energy.numel() != B or grad.numel() != B * self.n_exc:
            raise ValueError("theta [B, K], energy [B] and grad [B, K] do not match")
        st = stream if stream is not None else torch.cuda.current_stream(theta.device).cuda_stream
        check(lib().ucc_energy_grad_noalloc(self._h, _vp(theta.data_ptr()), B, _vp(energy.data_ptr()),
                                            _vp(grad.data_ptr()), _vp(st)), "ucc_energy_grad_noalloc")

    def energy_trotter_free(self, theta, stream=None, return_terms=False):
        """E [B] of the Trotter-free ansatz exp(sum_k theta_k G_k)|HF> (no product formula);
        with return_terms also the series terms used per entry (int32 [B])."""
        L = lib()
        if _is_torch_cuda(theta):
            import torch
            th = theta.detach().to(torch.float64).contiguous()
            B = th.numel() // self.n_exc
            if th.numel() != B * self.n_exc or B < 1:
                raise ValueError("theta must hold B * n_exc amplitudes")
            E = torch.empty(B, dtype=torch.float64, device=th.device)
            terms = np.zeros(B, dtype=np.int32)
            st = stream if stream is not None else torch.cuda.current_stream(th.device).cuda_stream
            check(L.ucc_energy_trotter_free(self._h, _vp(th.data_ptr()), B, _vp(E.data_ptr()),
                                            _ptr(terms), _vp(st)), "ucc_energy_trotter_free")
        else:
            th = np.ascontiguousarray(theta, dtype=np.float64)
            B = th.size // self.n_exc
            if th.size != B * self.n_exc or B < 1:
                raise ValueError("theta must hold B * n_exc amplitudes")
            E = np.empty(B)
            terms = np.zeros(B, dtype=np.int32)
            st = _vp(stream) if stream is not None else None
            check(L.ucc_energy_trotter_free(self._h, _ptr(th), B, _ptr(E), _ptr(terms), st),
                  "ucc_energy_trotter_free")
        return (E, terms) if return_terms else E

    def energy_grad_trotter_free(self, theta, stream=None, return_terms=False):
        """(E [B], dE/dtheta [B, K]) of the Trotter-free ansatz by the adjoint of the series;
        with return_terms also the series terms used per entry."""
        L = lib()
        if _is_torch_cuda(theta):
            import torch
            th = theta.detach().to(torch.float64).contiguous()
            B = th.numel() // self.n_exc
            if th.numel() != B * self.n_exc or B < 1:
                raise ValueError("theta must hold B * n_exc amplitudes")
            E = torch.empty(B, dtype=torch.float64, device=th.device)
            G = torch.empty(B, self.n_exc, dtype=torch.float64, device=th.device)
            terms = np.zeros(B, dtype=np.int32)
            st = stream if stream is not None else torch.cuda.current_stream(th.device).cuda_stream
            check(L.ucc_energy_grad_trotter_free(self._h, _vp(th.data_ptr()), B, _vp(E.data_ptr()),
                                                 _vp(G.data_ptr()), _ptr(terms), _vp(st)),
                  "ucc_energy_grad_trotter_free")
        else:
            th = np.ascontiguousarray(theta, dtype=np.float64)
            B = th.size // self.n_exc
            if th.size != B * self.n_exc or B < 1:
                raise ValueError("theta must hold B * n_exc amplitudes")
            E = np.empty(B)
            G = np.empty((B, self.n_exc))
            terms = np.zeros(B, dtype=np.int32)
            st = _vp(stream) if stream is not None else None
            check(L.ucc_energy_grad_trotter_free(self._h, _ptr(th), B, _ptr(E), _ptr(G), _ptr(terms), st),
                  "ucc_energy_grad_trotter_free")
        return (E, G, terms) if return_terms else (E, G)

    def generator_passes(self):
        """(local masks [n_passes] uint32, pass of each excitation [n_exc] int32) of the
        Trotter-free evaluation's generator plan."""
        L = lib()
        n = ctypes.c_int32()
        check(L.ucc_get_generator_passes(self._h, 0, None, None, ctypes.byref(n)),
              "ucc_get_generator_passes")
        local = np.zeros(max(n.value, 1), dtype=np.uint32)
        where = np.full(self.n_exc, -1, dtype=np.int32)
        check(L.ucc_get_generator_passes(self._h, n.value, _ptr(local), _ptr(where), ctypes.byref(n)),
              "ucc_get_generator_passes")
        return local[: n.value], where

    def partials_passes(self):
        """(local masks [n_windows] uint32, window of each factor [L] int32) of the order-free
        windows of the Trotter-free gradient's partials-only reverse passes."""
        L = lib()
        n = ctypes.c_int32()
        check(L.ucc_get_partials_passes(self._h, 0, None, None, ctypes.byref(n)),
              "ucc_get_partials_passes")
        info = self.plan_info()
        nf = self.n_exc * info["trotter_steps"] * info["trotter_order"]
        local = np.zeros(max(n.value, 1), dtype=np.uint32)
        where = np.full(nf, -1, dtype=np.int32)
        check(L.ucc_get_partials_passes(self._h, n.value, _ptr(local), _ptr(where), ctypes.byref(n)),
              "ucc_get_partials_passes")
        return local[: n.value], where

    def state(self, b=0):
        out = np.empty(2 << self.n_qubits)
        check(lib().ucc_get_state(self._h, int(b), _ptr(out)), "ucc_get_state")
        return out[0::2] + 1j * out[1::2]

    # ------------------------------------------------------------ profiling
    def profile(self, enable=True):
        """Bracket every later kernel launch with HIP events on the call's stream."""
        check(lib().ucc_profile(self._h, int(bool(enable))), "ucc_profile")

    def profile_read(self, reset=True):
        """{kind: dict(launches, ms, bytes)} accumulated since the last reset."""
        st = (KernelStat * N_KERNEL_KINDS)()
        check(lib().ucc_profile_read(self._h, st, int(bool(reset))), "ucc_profile_read")
        return {name: dict(launches=st[i].launches, ms=st[i].ms, bytes=st[i].bytes)
                for i, name in enumerate(KERNEL_KINDS)}

    # ------------------------------------------------------------ introspection
    def plan_info(self):
        info = PlanInfo()
        check(lib().ucc_get_plan_info(self._h, ctypes.byref(info)), "ucc_get_plan_info")
        d = {f: getattr(info, f) for f, _ in PlanInfo._fields_ if f != "perm"}
        d["perm"] = list(info.perm)[: info.n_qubits]
        return d

    def batch_compatible(self, other):
        """True if server jobs on this context and `other` share batched launches."""
        out = ctypes.c_int32()
        check(lib().ucc_batch_compatible(self._h, other._h, ctypes.byref(out)),
              "ucc_batch_compatible")
        return bool(out.value)

    def pauli_terms(self):
        n = self.plan_info()["n_pauli"]
        x, z, c = np.empty(n, np.uint64), np.empty(n, np.uint64), np.empty(n)
        check(lib().ucc_get_pauli_terms(self._h, _ptr(x), _ptr(z), _ptr(c)))
        return x, z, c

    def group_table(self):
        info = self.plan_info()
        G, n = info["n_groups"], info["state_qubits"]
        xm, m, valid = (np.empty(G, np.uint32) for _ in range(3))
        A = np.empty((G, 16))
        B = np.empty((G, 16, n))
        diag = np.empty(1 + n + n * n)
        check(lib().ucc_get_group_table(self._h, _ptr(xm), _ptr(m), _ptr(valid), _ptr(A), _ptr(B),
                                        _ptr(diag)))
        return dict(x=xm, m=m, valid=valid, A=A, B=B, c0=diag[0], a=diag[1:1 + n],
                    b=diag[1 + n:].reshape(n, n))

    def excitation_table(self):
        K = self.n_exc
        supp, frm, m = (np.empty(K, np.uint32) for _ in range(3))
        sig = np.empty(K, np.int32)
        check(lib().ucc_get_excitation_table(self._h, _ptr(supp), _ptr(frm), _ptr(m), _ptr(sig)))
        return dict(supp=supp, frm=frm, m=m, sigma=sig)

    def pass_table(self):
        info = self.plan_info()
        P = info["n_fwd_passes"] + info["n_exp_passes"] + info["n_rev_passes"]
        kind, first, count = (np.empty(P, np.int32) for _ in range(3))
        local = np.empty(P, np.uint32)
        L = self.n_exc * info["trotter_steps"] * info["trotter_order"]
        items = np.empty(2 * L + info["n_groups"], np.int32)
        check(lib().ucc_get_pass_table(self._h, _ptr(kind), _ptr(local), _ptr(first), _ptr(count),
                                       _ptr(items)))
        return [dict(kind=int(kind[i]), local=int(local[i]),
                     items=items[first[i]:first[i] + count[i]].copy()) for i in range(P)]

    # ------------------------------------------------------------ lifetime
    def close(self):
        if self._h:
            lib().ucc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Server:
    """Continuous-batching steepest-descent VQE server (ucc_server_* calls).

    submit(ctx, theta0, iters, lr) -> ticket; poll(ticket) -> None while running, else the
    result; wait(ticket) -> result.  A result is dict(status, energies [iters + 1],
    theta [n_exc], admit_s, done_s, rounds); a cancelled job has status UCC_ECANCELED.
    """

    def __init__(self, hbm_budget=0, slots=64, max_queue=0):
        h = _vp()
        check(lib().ucc_server_create(int(hbm_budget), int(slots), int(max_queue), ctypes.byref(h)),
              "ucc_server_create")
        self._h = h
        self._meta = {}

    def submit(self, ctx, theta0, iters, lr):
        th = np.ascontiguousarray(theta0, dtype=np.float64).reshape(-1)
        if th.size != ctx.n_exc:
            raise ValueError("theta0 must hold n_exc amplitudes")
        t = ctypes.c_uint64()
        check(lib().ucc_submit(self._h, ctx._h, _ptr(th), int(iters), float(lr), 0,
                               ctypes.byref(t)), "ucc_submit")
        self._meta[t.value] = (int(iters), ctx.n_exc)
        return t.value

    def _bufs(self, ticket):
        if ticket not in self._meta:  # not submitted here: the library reports the status
            return None, None, np.zeros(4)
        iters, K = self._meta[ticket]
        return np.empty(iters + 1), np.empty(K), np.empty(4)

    @staticmethod
    def _result(status, e, th, tm):
        rounds = int(tm[2])
        return dict(status=int(status), energies=e[:rounds].copy() if status else e, theta=th,
                    admit_s=float(tm[0]), done_s=float(tm[1]), rounds=rounds)

    def poll(self, ticket):
        done = ctypes.c_int32()
        e, th, tm = self._bufs(ticket)
        st = lib().ucc_poll(self._h, ticket, ctypes.byref(done), _ptr(e), _ptr(th), _ptr(tm))
        if not done.value:
            check(st, "ucc_poll")
            return None
        if st not in (0, STATUS_CODES["UCC_ECANCELED"]):
            check(st, "ucc_poll")
        return self._result(st, e, th, tm)

    def wait(self, ticket):
        e, th, tm = self._bufs(ticket)
        st = lib().ucc_wait(self._h, ticket, _ptr(e), _ptr(th), _ptr(tm))
        self._meta.pop(ticket, None)
        if st not in (0, STATUS_CODES["UCC_ECANCELED"]):
            check(st, "ucc_wait")
        return self._result(st, e, th, tm)

    def cancel(self, ticket):
        check(lib().ucc_cancel(self._h, ticket), "ucc_cancel")

    def close(self):
        if self._h:
            lib().ucc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _autograd():
    import torch

    class UCCEnergy(torch.autograd.Function):
        """E(theta) with dE/dtheta from the library's adjoint sweep.

        forward(theta [B, K] or [K] float64 CUDA tensor, ctx: Context) -> E [B] or scalar.
        """

        @staticmethod
        def forward(fctx, theta, ctx):
            E, G = ctx.energy_grad(theta)
            fctx.save_for_backward(G)
            fctx.scalar = theta.dim() == 1
            return E[0] if fctx.scalar else E

        @staticmethod
        def backward(fctx, gE):
            (G,) = fctx.saved_tensors
            if fctx.scalar:
                return gE * G[0], None
            return gE.unsqueeze(-1) * G, None

    return UCCEnergy


_UCCEnergy = None


def stream_probe(src, dst, nbytes, mode, stream=None):
    """ucc_stream_probe on torch CUDA tensors: mode 0 copies nbytes of src into dst, mode 1
    reads nbytes of src (dst receives per-workgroup sums; at least 64 KiB)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(src.device).cuda_stream
    check(lib().ucc_stream_probe(_vp(src.data_ptr()), _vp(dst.data_ptr()), int(nbytes), int(mode),
                                 _vp(st)), "ucc_stream_probe")


def fmo2_energy(e_mono, e_dimer):
    """Eq. 1: sum over pairs I > J of E_IJ minus (N_f - 2) times the sum of the E_I.  e_dimer
    lists the pairs (1,0), (2,0), (2,1), (3,0), ..."""
    em = np.ascontiguousarray(e_mono, dtype=np.float64)
    ed = np.ascontiguousarray(e_dimer, dtype=np.float64)
    if ed.size != em.size * (em.size - 1) // 2:
        raise ValueError("e_dimer must hold one energy per fragment pair")
    out = ctypes.c_double()
    check(lib().ucc_fmo2_energy(em.size, _ptr(em), _ptr(ed), ctypes.byref(out)), "ucc_fmo2_energy")
    return out.value


def ucc_energy_fn(theta, ctx):
    """Differentiable energy: torch autograd through the HIP adjoint gradient."""
    global _UCCEnergy
    if _UCCEnergy is None:
        _UCCEnergy = _autograd()
    return _UCCEnergy.apply(theta, ctx)
