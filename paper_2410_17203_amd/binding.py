"""Python binding of the C ABI in include/opf.h (ctypes; marshalling only).

PyTorch supplies the device workspace (one uint8 tensor) and the HIP stream;
every step of the iteration runs in the HIP library.  There is no fallback:
if libopf.so is missing or no GPU is visible the constructor raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_int32, c_int64,
                    c_size_t, c_void_p)
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("OPF_LIB", os.path.join(HERE, "_lib", "libopf.so"))
HEADER = os.path.join(os.path.dirname(HERE), "include", "opf.h")

F64, F32, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}

STATUS = {0: "OPF_OK", 1: "OPF_NOT_CONVERGED", -1: "OPF_E_INVALID", -2: "OPF_E_OOM",
          -3: "OPF_E_HIP", -4: "OPF_E_STATE", -5: "OPF_E_NUMERIC"}

FIELDS = {"P": 0, "TH1": 1, "TH2": 2, "V1": 3, "V2": 4, "U": 5, "PBAR": 6, "THBAR": 7,
          "PNC": 8, "THNC": 9, "VNC": 10}
KERNELS = ["devices", "sweep", "finalize", "rescale"]


class Options(Structure):
    _fields_ = [
        ("state_dtype", c_int32), ("dual_dtype", c_int32),
        ("rho_p", c_double), ("rho_theta", c_double),
        ("mu", c_double), ("gamma", c_double),
        ("adapt_every", c_int32),
        ("eps", c_double), ("eps_relative", c_int32),
        ("max_iter", c_int32), ("min_iter", c_int32),
        ("block_iters", c_int32), ("check_every", c_int32),
        ("inner_iters", c_int32), ("inner_omega_scale", c_double),
        ("polish_fp64", c_int32), ("polish_factor", c_double), ("use_graphs", c_int32),
        ("hip_stream", c_void_p),
        ("sweep_tiles", c_int32),
    ]


class Network(Structure):
    _fields_ = [
        ("N", c_int32), ("T", c_int32), ("K", c_int32),
        ("L", c_int32), ("line_from", POINTER(c_int32)), ("line_to", POINTER(c_int32)),
        ("line_sus", POINTER(c_double)), ("line_cap", POINTER(c_double)),
        ("outage", POINTER(c_int32)),
        ("G", c_int32), ("gen_node", POINTER(c_int32)),
        ("gen_c2", POINTER(c_double)), ("gen_c1", POINTER(c_double)),
        ("gen_pmin", POINTER(c_double)), ("gen_pmax", POINTER(c_double)),
        ("gen_ramp", POINTER(c_double)),
        ("D", c_int32), ("load_node", POINTER(c_int32)), ("load_d", POINTER(c_double)),
        ("B", c_int32), ("bat_node", POINTER(c_int32)),
        ("bat_P", POINTER(c_double)), ("bat_dur", POINTER(c_double)),
        ("bat_eta", POINTER(c_double)), ("bat_alpha", POINTER(c_double)),
        ("line_kind", POINTER(c_int32)),
        ("n_chg", c_int32), ("chg_k", POINTER(c_int32)), ("chg_line", POINTER(c_int32)),
        ("chg_sus", POINTER(c_double)), ("chg_cap", POINTER(c_double)),
    ]


class Resid(Structure):
    _fields_ = [
        ("iter", c_int64),
        ("primal_p", c_double), ("primal_theta", c_double),
        ("dual_p", c_double), ("dual_theta", c_double),
        ("rms_primal", c_double), ("rms_dual", c_double),
        ("threshold", c_double), ("objective", c_double),
        ("rho_p", c_double), ("rho_theta", c_double),
        ("converged", c_int32), ("precision", c_int32),
    ]

    def as_dict(self) -> Dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Tuning(Structure):
    _fields_ = [("lanes_shift", c_int32), ("grid_factor", c_double),
                ("ms_per_iter", c_double), ("from_cache", c_int32), ("tiled", c_int32),
                ("tile_groups", c_int32)]


class Layout(Structure):
    _fields_ = [("N", c_int32), ("T", c_int32), ("K", c_int32), ("Kpp", c_int32),
                ("L", c_int32), ("Jnc", c_int32), ("state_dtype", c_int32),
                ("dual_dtype", c_int32), ("chunk", c_int32),
                *[(n, c_size_t) for n in ["P", "Tm", "V1", "V2", "Td", "U", "W", "TB", "pnc",
                                          "thnc", "vbar"]],
                ("Ldc", c_int32), ("Hd", c_size_t), ("Zc", c_int32), ("Tz", c_size_t)]


class OpfError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libopf.so and declares every entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OpfError(f"{path} not built; run paper_2410_17203_amd.build.build()")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "opf_default_options": (None, [POINTER(Options)]),
        "opf_create": (c_int32, [POINTER(Options), POINTER(c_void_p)]),
        "opf_check_network": (c_int32, [POINTER(Network), POINTER(Options), POINTER(c_int32)]),
        "opf_workspace_size": (c_int32, [P, POINTER(Network), POINTER(c_size_t)]),
        "opf_load_network": (c_int32, [P, POINTER(Network), c_void_p, c_size_t]),
        "opf_load_network_static": (c_int32, [P, POINTER(Network)]),
        "opf_iterate": (c_int32, [P, c_int32]),
        "opf_solve": (c_int32, [P, POINTER(Resid)]),
        "opf_residuals": (c_int32, [P, POINTER(Resid)]),
        "opf_residual_history": (c_int32, [P, POINTER(Resid), c_int32, POINTER(c_int32)]),
        "opf_field_size": (c_int32, [P, c_int32, POINTER(c_size_t)]),
        "opf_get_field": (c_int32, [P, c_int32, c_void_p, c_size_t]),
        "opf_set_timing": (c_int32, [P, c_int32]),
        "opf_kernel_times": (c_int32, [P, POINTER(c_double), POINTER(c_int64)]),
        "opf_kernel_bytes": (c_int32, [P, c_int32, POINTER(c_double)]),
        "opf_workspace_size_batch": (c_int32, [P, POINTER(Network), c_int32, POINTER(c_size_t)]),
        "opf_load_batch": (c_int32, [P, POINTER(Network), c_int32, c_void_p, c_size_t]),
        "opf_num_instances": (c_int32, [P, POINTER(c_int32)]),
        "opf_reset": (c_int32, [P]),
        "opf_residuals_i": (c_int32, [P, c_int32, POINTER(Resid)]),
        "opf_residual_history_i": (c_int32, [P, c_int32, POINTER(Resid), c_int32, POINTER(c_int32)]),
        "opf_field_size_i": (c_int32, [P, c_int32, c_int32, POINTER(c_size_t)]),
        "opf_get_field_i": (c_int32, [P, c_int32, c_int32, c_void_p, c_size_t]),
        "opf_autotune": (c_int32, [P, c_int32, c_char_p, POINTER(Tuning)]),
        "opf_state_layout": (c_int32, [P, c_int32, POINTER(Layout)]),
        "opf_state_size": (c_int32, [P, POINTER(c_size_t)]),
        "opf_get_state": (c_int32, [P, c_void_p, c_size_t]),
        "opf_set_state": (c_int32, [P, c_void_p, c_size_t]),
        "opf_tape_workspace_size": (c_int32, [P, c_int32, c_int32, POINTER(c_size_t)]),
        "opf_tape_forward": (c_int32, [P, c_int32, c_int32, c_void_p, c_size_t]),
        "opf_tape_forward_warm": (c_int32, [P, c_int32, c_int32, c_int32, c_void_p, c_size_t,
                                            POINTER(c_int32)]),
        "opf_adjoint": (c_int32, [P, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
        "opf_last_error": (c_char_p, [P]),
        "opf_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_options() -> Options:
    o = Options()
    load_library().opf_default_options(byref(o))
    return o


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class NetworkArrays:
    """Keeps the marshalled host arrays alive for the lifetime of a call."""

    def __init__(self, inst):
        i32, f64 = np.int32, np.float64
        T = int(inst.T)
        self.keep = []

        def p(a, dt, ctype):
            a = _arr(a, dt)
            self.keep.append(a)
            return a.ctypes.data_as(POINTER(ctype))

        n = Network()
        n.N, n.T, n.K = int(inst.N), T, int(inst.K)
        n.L = len(inst.line_from)
        n.line_from = p(inst.line_from, i32, c_int32)
        n.line_to = p(inst.line_to, i32, c_int32)
        n.line_sus = p(inst.line_sus, f64, c_double)
        n.line_cap = p(inst.line_cap, f64, c_double)
        n.outage = p(inst.outage, i32, c_int32)
        n.G = len(inst.gen_node)
        n.gen_node = p(inst.gen_node, i32, c_int32)
        n.gen_c2 = p(inst.gen_c2, f64, c_double)
        n.gen_c1 = p(inst.gen_c1, f64, c_double)
        n.gen_pmin = p(np.reshape(inst.gen_pmin, (n.G, T)), f64, c_double)
        n.gen_pmax = p(np.reshape(inst.gen_pmax, (n.G, T)), f64, c_double)
        n.gen_ramp = p(inst.gen_ramp, f64, c_double)
        n.D = len(inst.load_node)
        n.load_node = p(inst.load_node, i32, c_int32)
        n.load_d = p(np.reshape(inst.load_d, (n.D, T)), f64, c_double)
        n.B = len(inst.bat_node)
        n.bat_node = p(inst.bat_node, i32, c_int32)
        n.bat_P = p(inst.bat_P, f64, c_double)
        n.bat_dur = p(inst.bat_dur, f64, c_double)
        n.bat_eta = p(inst.bat_eta, f64, c_double)
        n.bat_alpha = p(inst.bat_alpha, f64, c_double)
        kind = getattr(inst, "line_kind", None)
        if kind is not None:
            n.line_kind = p(kind, i32, c_int32)
        ck = getattr(inst, "chg_k", None)
        if ck is not None and len(ck):
            n.n_chg = len(ck)
            n.chg_k = p(ck, i32, c_int32)
            n.chg_line = p(inst.chg_line, i32, c_int32)
            n.chg_sus = p(inst.chg_sus, f64, c_double)
            n.chg_cap = p(inst.chg_cap, f64, c_double)
        self.net = n


def _options(dtype: str, dual_dtype: Optional[str], stream_ptr: int, **kw) -> Options:
    o = default_options()
    o.state_dtype = DTYPES[dtype]
    o.dual_dtype = DTYPES[dual_dtype] if dual_dtype else DTYPES[dtype]
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, float(v) if isinstance(getattr(o, k), float) else int(v))
    o.hip_stream = c_void_p(stream_ptr)
    return o


def check_network(inst, dtype: str = "f64", dual_dtype: Optional[str] = None, **opts) -> bool:
    """Host-only check of one network (opf_check_network): raises OpfError
    with the library's reason if it would be rejected, else returns whether
    the tiled sweep's clusters exist.  Needs no GPU."""
    lib = load_library()
    arrays = NetworkArrays(inst)
    o = _options(dtype, dual_dtype, 0, **opts)
    tiled = c_int32(-1)
    st = lib.opf_check_network(byref(arrays.net), byref(o), byref(tiled))
    if st != 0:
        raise OpfError(f"{st}: {lib.opf_last_error(None).decode()}")
    return bool(tiled.value)


class Solver:
    """One instance, or a batch of instances, loaded on one GPU.

    inst: one network, or a list of networks (a batch: every phase of an
    iteration is one launch over all of them).  dtype: 'f64' or 'f32'
    iterate; dual_dtype 'bf16' stores the line phase duals in BF16 (with
    dtype 'f32').  Keyword options map onto opf_options.
    """

    def __init__(self, inst, dtype: str = "f64", dual_dtype: Optional[str] = None,
                 device: str = "cuda:0", static_workspace: bool = False, **opts):
        import torch
        if not torch.cuda.is_available():
            raise OpfError("no GPU visible: the HIP library has no CPU path")
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.opt = _options(dtype, dual_dtype, self.stream.cuda_stream, **opts)
        ctx = c_void_p()
        self._check(self.lib.opf_create(byref(self.opt), byref(ctx)), None)
        self.ctx = ctx
        self.ws = None
        self.load(inst, static_workspace)

    def load(self, inst, static_workspace: bool = False):
        """(Re)loads the context with one network or a batch, resetting the
        iterate.  static_workspace: use the library's fixed per-device
        workspace (opf_load_network_static; one network, nothing allocated)
        instead of a new device tensor."""
        torch = self.torch
        insts = list(inst) if isinstance(inst, (list, tuple)) else [inst]
        arrays = [NetworkArrays(x) for x in insts]
        nets = (Network * len(insts))(*[a.net for a in arrays])
        nbytes = c_size_t()
        self._check(self.lib.opf_workspace_size_batch(self.ctx, nets, len(insts), byref(nbytes)))
        if static_workspace:
            if len(insts) != 1:
                raise OpfError("the fixed workspace holds one instance, not a batch")
            self._check(self.lib.opf_load_network_static(self.ctx, nets))
            self.ws = None
        else:
            ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self._check(self.lib.opf_load_batch(self.ctx, nets, len(insts),
                                                c_void_p(ws.data_ptr()), nbytes))
            self.ws = ws
        self.insts = insts
        self.workspace_bytes = int(nbytes.value)
        self.shapes = [dict(N=int(x.N), T=int(x.T), K=int(x.K), L=len(x.line_from),
                            Jnc=len(x.gen_node) + len(x.load_node) + len(x.bat_node))
                       for x in insts]
        s0 = self.shapes[0]
        self.N, self.T, self.K, self.L, self.Jnc = s0["N"], s0["T"], s0["K"], s0["L"], s0["Jnc"]

    # -- helpers ---------------------------------------------------------------
    def _check(self, st, ctx="self"):
        if st in (0, 1):
            return st
        c = self.ctx if ctx == "self" else None
        msg = self.lib.opf_last_error(c)
        raise OpfError(f"{STATUS.get(st, st)}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "ctx", None) is not None:
            self.lib.opf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_instances(self) -> int:
        return len(self.shapes)

    # -- iteration ---------------------------------------------------------------
    def iterate(self, n: int):
        self._check(self.lib.opf_iterate(self.ctx, int(n)))

    def solve(self) -> Dict:
        r = Resid()
        st = self._check(self.lib.opf_solve(self.ctx, byref(r)))
        d = r.as_dict()
        d["status"] = STATUS[st]
        return d

    def reset(self):
        self._check(self.lib.opf_reset(self.ctx))

    def residuals(self, instance: int = 0) -> Dict:
        r = Resid()
        self._check(self.lib.opf_residuals_i(self.ctx, int(instance), byref(r)))
        return r.as_dict()

    def history(self, max_records: int = 4096, instance: int = 0) -> List[Dict]:
        buf = (Resid * max_records)()
        n = c_int32()
        self._check(self.lib.opf_residual_history_i(self.ctx, int(instance), buf, max_records,
                                                    byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    def synchronize(self):
        self.stream.synchronize()

    # -- the iterate: zero-copy views, export, warm start ----------------------
    def layout(self, instance: int = 0) -> Dict:
        lay = Layout()
        self._check(self.lib.opf_state_layout(self.ctx, int(instance), byref(lay)))
        return {name: getattr(lay, name) for name, _ in lay._fields_}

    def view(self, name: str, instance: int = 0):
        """Zero-copy views of one array of the current iterate, valid until
        the next iteration.  Line and node arrays: a list with one [T, count,
        w] tensor per chunk of contingencies (layout()['chunk'] wide, the last one
        narrower); Hd (DC links) likewise over layout()['Ldc'] links; Td [T, Kpp];
        Tz [T, Zc] (lines taken out by changes);
        device arrays [Jnc, T]."""
        torch = self.torch
        if self.ws is None:
            raise OpfError("zero-copy views need a caller workspace, not the fixed one")
        lay = self.layout(instance)
        dt = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}
        is_dual = name in ("V1", "V2")
        dtype = dt[lay["dual_dtype"] if is_dual else lay["state_dtype"]]
        T, L, N, Kpp, J = lay["T"], lay["L"], lay["N"], lay["Kpp"], lay["Jnc"]
        esize = torch.empty((), dtype=dtype).element_size()
        off = lay[name] // esize
        if name in ("Td", "Tz", "pnc", "thnc", "vbar"):
            shape = {"Td": (T, Kpp), "Tz": (T, lay["Zc"])}.get(name, (J, T))
            n = int(np.prod(shape))
            return self.ws[lay[name]:lay[name] + n * esize].view(dtype).view(shape)
        count = {"P": L, "Tm": L, "V1": L, "V2": L, "Hd": lay["Ldc"]}.get(name, N)
        flat = self.ws.view(dtype) if self.ws.numel() % esize == 0 else None
        out = []
        ch = lay["chunk"]
        for c0 in range(0, Kpp, ch):
            w = min(ch, Kpp - c0)
            out.append(flat.as_strided((T, count, w), (Kpp * count, w, 1), off + c0 * count))
        return out

    def get_state(self):
        """The whole iterate and penalties as a uint8 device tensor."""
        torch = self.torch
        nbytes = c_size_t()
        self._check(self.lib.opf_state_size(self.ctx, byref(nbytes)))
        out = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self._check(self.lib.opf_get_state(self.ctx, c_void_p(out.data_ptr()), nbytes))
        return out

    def set_state(self, blob):
        """Warm start from a blob returned by get_state (same network shape)."""
        blob = blob.contiguous()
        self.torch.cuda.current_stream(self.device).synchronize()
        self._check(self.lib.opf_set_state(self.ctx, c_void_p(blob.data_ptr()),
                                           c_size_t(blob.numel())))

    # -- derivatives through unrolled iterations ------------------------------
    def checkpoint_interval(self, n_iters: int, budget_frac: float = 0.25) -> int:
        """The smallest checkpoint interval among 1, 2, 5, 10, 25, 50 whose
        tape for n_iters iterations fits in budget_frac of the device's free
        memory (50 if none does).  Interval 1 keeps every iterate, so the
        adjoint recomputes nothing."""
        free, _ = self.torch.cuda.mem_get_info(self.device)
        nbytes = c_size_t()
        for every in (1, 2, 5, 10, 25, 50):
            self._check(self.lib.opf_tape_workspace_size(self.ctx, int(n_iters), every,
                                                         byref(nbytes)))
            if nbytes.value <= budget_frac * free:
                return every
        return 50

    def tape_forward(self, n_iters: int, checkpoint_every: Optional[int] = None) -> Dict:
        """Runs exactly n_iters iterations from the zero start, recording what
        the adjoint needs; returns the residual record of the last one.
        checkpoint_every None: checkpoint_interval(n_iters)."""
        torch = self.torch
        if checkpoint_every is None:
            checkpoint_every = self.checkpoint_interval(n_iters)
        self.tape_every = int(checkpoint_every)
        nbytes = c_size_t()
        self._check(self.lib.opf_tape_workspace_size(self.ctx, int(n_iters),
                                                     int(checkpoint_every), byref(nbytes)))
        self.tape = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        self._check(self.lib.opf_tape_forward(self.ctx, int(n_iters), int(checkpoint_every),
                                              c_void_p(self.tape.data_ptr()), nbytes))
        return self.residuals()

    def tape_forward_warm(self, min_iters: int, max_iters: int, checkpoint_every: int = 50):
        """Records a run from the current iterate until the stopping rule holds
        (at least min_iters, at most max_iters iterations); returns the last
        residual record and the number of iterations run."""
        torch = self.torch
        nbytes = c_size_t()
        self._check(self.lib.opf_tape_workspace_size(self.ctx, int(max_iters),
                                                     int(checkpoint_every), byref(nbytes)))
        self.tape = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        n = c_int32()
        self._check(self.lib.opf_tape_forward_warm(self.ctx, int(min_iters), int(max_iters),
                                                   int(checkpoint_every),
                                                   c_void_p(self.tape.data_ptr()), nbytes,
                                                   byref(n)))
        return self.residuals(), int(n.value)

    def adjoint(self, cot_power=None, cot_objective: float = 0.0) -> Dict:
        """Reverse pass of the recorded run.  cot_power: [G+D+B, T] weights on
        the final device powers (or None); cot_objective: weight of the final
        objective.  Returns float64 device tensors: 'load' [D, T], 'cap' [L],
        'pmax' [G, T] (derivatives w.r.t. demand, line capacity, generator
        upper limit)."""
        torch = self.torch
        inst = self.insts[0]
        G, D, T, L = len(inst.gen_node), len(inst.load_node), int(inst.T), len(inst.line_from)
        f64 = dict(dtype=torch.float64, device=self.device)
        cot = None
        if cot_power is not None:
            cot = torch.as_tensor(cot_power, **f64).reshape(self.Jnc, T).contiguous()
        out = {"load": torch.zeros(D, T, **f64), "cap": torch.zeros(L, **f64),
               "pmax": torch.zeros(G, T, **f64)}
        torch.cuda.current_stream(self.device).synchronize()

        def ptr(x):
            return c_void_p(x.data_ptr()) if x is not None and x.numel() > 0 else None
        self._check(self.lib.opf_adjoint(self.ctx, ptr(cot), float(cot_objective),
                                         ptr(out["load"]), ptr(out["cap"]), ptr(out["pmax"])))
        return out

    def autotune(self, trials: int = 5, cache_path: Optional[str] = None) -> Dict:
        t = Tuning()
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.opf_autotune(self.ctx, int(trials), path, byref(t)))
        return {name: getattr(t, name) for name, _ in t._fields_}

    # -- state -------------------------------------------------------------------
    def field_device(self, name: str, instance: int = 0):
        """One field of the iterate as a float64 device tensor in the paper's
        layout ([K+1][L][T], [K+1][N][T] or [G+D+B][T])."""
        torch = self.torch
        fid = FIELDS[name]
        cnt = c_size_t()
        self._check(self.lib.opf_field_size_i(self.ctx, int(instance), fid, byref(cnt)))
        out = torch.empty(int(cnt.value), dtype=torch.float64, device=self.device)
        self._check(self.lib.opf_get_field_i(self.ctx, int(instance), fid,
                                             c_void_p(out.data_ptr()), cnt))
        self.stream.synchronize()
        s = self.shapes[instance]
        Kp = s["K"] + 1
        shape = {0: (Kp, s["L"], s["T"]), 5: (Kp, s["N"], s["T"]), 8: (s["Jnc"], s["T"])}
        key = 0 if fid <= 4 else (5 if fid <= 7 else 8)
        return out.reshape(shape[key])

    def field(self, name: str, instance: int = 0):
        """One field of the iterate as a float64 CPU tensor."""
        return self.field_device(name, instance).cpu()

    def state(self, instance: int = 0) -> Dict:
        return {k: self.field(k, instance) for k in FIELDS}

    # -- timing --------------------------------------------------------------------
    def set_timing(self, enable: bool):
        self._check(self.lib.opf_set_timing(self.ctx, 1 if enable else 0))

    def kernel_times(self) -> Dict[str, Dict]:
        ms = (c_double * 4)()
        n = (c_int64 * 4)()
        self._check(self.lib.opf_kernel_times(self.ctx, ms, n))
        return {KERNELS[i]: {"ms": ms[i], "launches": n[i]} for i in range(4)}

    def kernel_bytes(self, kernel: str) -> float:
        b = c_double()
        self._check(self.lib.opf_kernel_bytes(self.ctx, KERNELS.index(kernel), byref(b)))
        return b.value


def header_functions(path: str = HEADER) -> List[str]:
    """Names of the functions include/opf.h declares."""
    import re
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(opf_[a-z_]+)\s*\(", txt)))
