"""Python binding of the MI355X exact minimum-cut library (libmincut.so).

Argument marshalling only: graphs are handed to the C ABI of
include/mincut.h and include/mincut_steps.h as raw pointers; PyTorch supplies
device memory (workspaces, device copies of inputs) and the HIP stream. Every
step of the computation runs in the library's HIP kernels. If the library is
missing, importing the binding's entry points raises -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmincut.so")

MC_HOST, MC_DEVICE = 0, 1
MC_CF_PRIVATE, MC_CF_SHARED, MC_CF_AUTO = 0, 1, 2
CF_SHARED, CF_SEQUENTIAL, CF_PRIVATE, CF_LEVELS = 0, 1, 2, 3  # step modes
STATUS = {0: "MC_OK", -1: "MC_E_INVALID_ARG", -2: "MC_E_BAD_GRAPH", -3: "MC_E_OVERFLOW", -4: "MC_E_OOM",
          -5: "MC_E_DEVICE", -6: "MC_E_NOT_READY", -7: "MC_E_CANCELLED", -8: "MC_E_TIMEOUT"}
INT64_MAX = (1 << 63) - 1


class MincutError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("location", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("heuristic_min_n", ctypes.c_int32), ("lp_iters", ctypes.c_int32),
                ("pr_tri_deg_cap", ctypes.c_int32), ("capforest_passes", ctypes.c_int32),
                ("pass_len_cap", ctypes.c_int32), ("capforest_mode", ctypes.c_int32),
                ("levels_min_n", ctypes.c_int32), ("deterministic", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("batch_pass_threads", ctypes.c_int32), ("batch_lp", ctypes.c_int32),
                ("finish_max_n", ctypes.c_int32), ("queue", ctypes.c_int32), ("contract_mode", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("heuristic_levels", ctypes.c_int32),
                ("lambda_min_degree", ctypes.c_int64), ("lambda_heuristic", ctypes.c_int64),
                ("marks_pr", ctypes.c_int64), ("marks_capforest", ctypes.c_int64),
                ("fallback_passes", ctypes.c_int32), ("n_input", ctypes.c_int32), ("m_input", ctypes.c_int64),
                ("ms_total", ctypes.c_double), ("rounds_pr_only", ctypes.c_int32), ("input_normal", ctypes.c_int32),
                ("marks_tri", ctypes.c_int64), ("finish_rounds", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


MC_TUNE_MAX = 16


class Tuning(ctypes.Structure):
    _fields_ = [("pass_threads", ctypes.c_int32), ("lp", ctypes.c_int32), ("sample", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("cand_threads", ctypes.c_int32 * MC_TUNE_MAX),
                ("cand_lp", ctypes.c_int32 * MC_TUNE_MAX), ("cand_ms", ctypes.c_double * MC_TUNE_MAX),
                ("finish_max_n", ctypes.c_int32), ("queue", ctypes.c_int32),
                ("cand_finish", ctypes.c_int32 * MC_TUNE_MAX), ("cand_queue", ctypes.c_int32 * MC_TUNE_MAX)]


class RoundTime(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_in", ctypes.c_int32), ("m_in", ctypes.c_int64),
                ("n_out", ctypes.c_int32), ("m_out", ctypes.c_int64), ("ms", ctypes.c_double)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


MC_K_COUNT = 12  # kernels mc_profile times (MC_K_* in include/mincut.h)


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32), ("max_request_n", ctypes.c_int32),
                ("max_request_nnz", ctypes.c_int64), ("solo_min_n", ctypes.c_int32), ("solo_slots", ctypes.c_int32),
                ("deadline_ms", ctypes.c_double)]


class ReqStats(ctypes.Structure):
    _fields_ = [("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
                ("rounds", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DGraphC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("cap", ctypes.c_int64), ("off", ctypes.c_void_p), ("len", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("deg", ctypes.c_void_p)]


# name -> (restype, argtypes) for every symbol the headers declare
P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
SIGNATURES = {
    "mc_default_options": (None, [P]),
    "mc_ctx_create": (ctypes.c_int, [ctypes.c_int, P, P, P]),
    "mc_ctx_destroy": (ctypes.c_int, [P]),
    "mc_ctx_set_options": (ctypes.c_int, [P, P]),
    "mc_workspace_size": (ctypes.c_int, [P, I32, I32, P]),
    "mc_mincut": (ctypes.c_int, [P, P, P, SZ, P, P, P]),
    "mc_mincut_static": (ctypes.c_int, [P, P, P, P, P]),
    "mc_last_error": (ctypes.c_char_p, []),
    "mc_check_graph": (ctypes.c_int, [P, I32]),
    "mc_batch_workspace_size": (ctypes.c_int, [P, I32, P, P]),
    "mc_mincut_batch": (ctypes.c_int, [P, I32, P, P, SZ, P, P, P]),
    "mc_batch_autotune": (ctypes.c_int, [P, I32, P, P, SZ, I32, P]),
    "mc_server_create": (ctypes.c_int, [P, P, P]),
    "mc_server_destroy": (ctypes.c_int, [P]),
    "mc_server_submit": (ctypes.c_int, [P, P, P]),
    "mc_server_step": (ctypes.c_int, [P, P, P]),
    "mc_server_poll": (ctypes.c_int, [P, ctypes.c_uint64, P, P, P]),
    "mc_server_cancel": (ctypes.c_int, [P, ctypes.c_uint64]),
    "mc_server_state": (ctypes.c_int, [P, ctypes.c_uint64, P]),
    "mc_server_capacity": (ctypes.c_int, [P, P, P, P, P]),
    "mc_profile": (ctypes.c_int, [P, I32]),
    "mc_profile_read": (ctypes.c_int, [P, I32, P]),
    "mc_profile_round": (ctypes.c_int, [P, I32, P, P]),
    "mc_step_ws_size": (ctypes.c_int, [I32, I64, I32, P]),
    "mc_step_contract": (ctypes.c_int, [P, P, P, I32, P, P, SZ, P, P]),
    "mc_step_components": (ctypes.c_int, [P, I32, I64, P, P, P, P, P, SZ]),
    "mc_step_pr12": (ctypes.c_int, [P, P, I64, P, P, P, P, P, SZ]),
    "mc_step_lp": (ctypes.c_int, [P, P, P, P, P, SZ]),
    "mc_step_pr34": (ctypes.c_int, [P, P, I64, I32, P, P, P, P, P, P, SZ]),
    "mc_step_capforest": (ctypes.c_int, [P, P, I64, I32, I32, I32, I32, I32, P, P, P, P, P, P, P, P, SZ]),
}

_lib = None


def lib():
    """Load libmincut.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmincut.so is not built: run __graft_entry__.build() "
                              "or python paper_2609_07204_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise MincutError(rc, lib().mc_last_error().decode())


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def default_options(**kw):
    o = Options()
    lib().mc_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """A library context bound to one GPU and the current torch stream."""

    def __init__(self, device=0, stream=None, **options):
        torch = _torch()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.options = default_options(**options)
        h = ctypes.c_void_p()
        _check(lib().mc_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self.options),
                                   ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().mc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, **kw):
        o = Options()
        ctypes.pointer(o)[0] = self.options
        for k, v in kw.items():
            setattr(o, k, v)
        _check(lib().mc_ctx_set_options(self.h, ctypes.byref(o)))
        self.options = o

    # ------------------------------------------------------------ solve
    def workspace_bytes(self, n, nnz):
        b = ctypes.c_size_t()
        _check(lib().mc_workspace_size(self.h, n, nnz, ctypes.byref(b)))
        return b.value

    def upload(self, g):
        """Device copies (row_ptr, col, w) of a host graph."""
        torch = _torch()
        return (torch.as_tensor(np.ascontiguousarray(g.row_ptr, np.int32)).to(self.device),
                torch.as_tensor(np.ascontiguousarray(g.col, np.int32)).to(self.device),
                torch.as_tensor(np.ascontiguousarray(g.w, np.int64)).to(self.device))

    def mincut(self, g=None, dev=None, n=None, workspace=None, want_side=True, return_stats=False):
        """Minimum cut of a graph given either as a host graph `g` (fields
        n, row_ptr, col, w as numpy arrays) or as device tensors
        dev = (row_ptr, col, w) with n vertices. Returns (lambda, side) and,
        with return_stats, the mc_stats record as a dict."""
        torch = _torch()
        if dev is not None:
            rp, col, w = dev
            n = int(rp.numel() - 1)
            nnz = int(col.numel())
            csr = CSR(n, nnz, rp.data_ptr(), col.data_ptr() if nnz else 0, w.data_ptr() if nnz else 0, MC_DEVICE)
            keep = (rp, col, w)
        else:
            rp = np.ascontiguousarray(g.row_ptr, np.int32)
            col = np.ascontiguousarray(g.col, np.int32)
            w = np.ascontiguousarray(g.w, np.int64)
            n, nnz = int(g.n), int(rp[-1])
            csr = CSR(n, nnz, rp.ctypes.data, col.ctypes.data if nnz else 0, w.ctypes.data if nnz else 0, MC_HOST)
            keep = (rp, col, w)
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(n, nnz), dtype=torch.uint8, device=self.device)
        lam = ctypes.c_int64()
        side = np.zeros(n, np.uint8) if want_side else None
        st = Stats()
        _check(lib().mc_mincut(self.h, ctypes.byref(csr), ctypes.c_void_p(workspace.data_ptr()),
                               workspace.numel(), ctypes.byref(lam),
                               side.ctypes.data if want_side else None, ctypes.byref(st)))
        del keep
        if return_stats:
            return lam.value, side, st.as_dict()
        return lam.value, side

    # ------------------------------------------------------------ batch
    def _csr_array(self, graphs=None, devs=None):
        """ctypes array of mc_csr for host graphs or device (rp, col, w)
        tuples, and the objects that must stay alive while it is used."""
        keep = []
        if devs is not None:
            arr = (CSR * len(devs))()
            for i, (rp, col, w) in enumerate(devs):
                nnz = int(col.numel())
                arr[i] = CSR(int(rp.numel() - 1), nnz, rp.data_ptr(), col.data_ptr() if nnz else 0,
                             w.data_ptr() if nnz else 0, MC_DEVICE)
                keep.append((rp, col, w))
        else:
            arr = (CSR * len(graphs))()
            for i, g in enumerate(graphs):
                rp = np.ascontiguousarray(g.row_ptr, np.int32)
                col = np.ascontiguousarray(g.col, np.int32)
                w = np.ascontiguousarray(g.w, np.int64)
                nnz = int(rp[-1])
                arr[i] = CSR(int(g.n), nnz, rp.ctypes.data, col.ctypes.data if nnz else 0,
                             w.ctypes.data if nnz else 0, MC_HOST)
                keep.append((rp, col, w))
        return arr, keep

    def batch_workspace_bytes(self, graphs=None, devs=None):
        arr, keep = self._csr_array(graphs, devs)
        b = ctypes.c_size_t()
        _check(lib().mc_batch_workspace_size(self.h, len(arr), arr, ctypes.byref(b)))
        return b.value

    def mincut_batch(self, graphs=None, devs=None, workspace=None, want_sides=True, per_graph=False):
        """Minimum cuts of many graphs in one call (mc_mincut_batch): host
        graphs or device (rp, col, w) tuples. Returns (lambdas, sides), or
        (lambdas, sides, statuses) with per_graph=True, where a graph that
        fails its own checks gets its status and is skipped."""
        torch = _torch()
        arr, keep = self._csr_array(graphs, devs)
        k = len(arr)
        if workspace is None:
            b = ctypes.c_size_t()
            _check(lib().mc_batch_workspace_size(self.h, k, arr, ctypes.byref(b)))
            workspace = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        lams = np.zeros(k, np.int64)
        sides = [np.zeros(max(int(arr[i].n), 0), np.uint8) for i in range(k)] if want_sides else None
        sp = (ctypes.c_void_p * k)(*[s.ctypes.data for s in sides]) if want_sides else None
        st = np.zeros(k, np.int32) if per_graph else None
        _check(lib().mc_mincut_batch(self.h, k, arr, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                     lams.ctypes.data, sp, st.ctypes.data if per_graph else None))
        del keep
        return (lams, sides, st) if per_graph else (lams, sides)

    def batch_autotune(self, graphs=None, devs=None, workspace=None, sample=0):
        """Time the batched form on a spread sample of the batch under every
        pass workgroup size, with and without the admission bound, then the
        finisher's size limit and queue, and keep the fastest in this context
        (mc_batch_autotune). Returns the timings."""
        torch = _torch()
        arr, keep = self._csr_array(graphs, devs)
        k = len(arr)
        if workspace is None:
            b = ctypes.c_size_t()
            _check(lib().mc_batch_workspace_size(self.h, k, arr, ctypes.byref(b)))
            workspace = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        t = Tuning()
        _check(lib().mc_batch_autotune(self.h, k, arr, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                       int(sample), ctypes.byref(t)))
        del keep
        self.options.batch_pass_threads = t.pass_threads
        self.options.batch_lp = t.lp
        self.options.finish_max_n = t.finish_max_n
        self.options.queue = t.queue
        return {"pass_threads": t.pass_threads, "lp": t.lp, "finish_max_n": t.finish_max_n, "queue": t.queue,
                "sample": t.sample,
                "candidates": [{"pass_threads": t.cand_threads[i], "lp": t.cand_lp[i],
                                "finish_max_n": t.cand_finish[i], "queue": t.cand_queue[i], "ms": t.cand_ms[i]}
                               for i in range(t.candidates)]}

    # ------------------------------------------------------------ timing
    def profile(self, on=True):
        """Switch kernel timing on (zeroing the totals) or off."""
        _check(lib().mc_profile(self.h, int(bool(on))))

    def profile_rounds(self):
        """Rounds of the last solve made while timing was on (mc_profile_round):
        [{"kind": "exact" | "level" | "coarse", "n_in", "m_in", "n_out", "m_out", "ms"}]."""
        cnt = ctypes.c_int32()
        _check(lib().mc_profile_round(self.h, 0, None, ctypes.byref(cnt)))
        kinds = {0: "exact", 1: "level", 2: "coarse"}
        out = []
        for i in range(cnt.value):
            r = RoundTime()
            _check(lib().mc_profile_round(self.h, i, ctypes.byref(r), ctypes.byref(cnt)))
            out.append({"kind": kinds.get(r.kind, str(r.kind)), "n_in": r.n_in, "m_in": r.m_in, "n_out": r.n_out,
                        "m_out": r.m_out, "ms": r.ms})
        return out

    def profile_read(self):
        """{kernel name: {"launches", "ms", "bytes"}} since profiling was switched on."""
        out = {}
        for k in range(MC_K_COUNT):
            kt = KernelTime()
            _check(lib().mc_profile_read(self.h, k, ctypes.byref(kt)))
            out[kt.name.decode()] = {"launches": kt.launches, "ms": kt.ms, "bytes": kt.bytes}
        return out

    # ------------------------------------------------------------ steps
    def step_workspace(self, n, cap, passes=1):
        b = ctypes.c_size_t()
        _check(lib().mc_step_ws_size(n, cap, passes, ctypes.byref(b)))
        return _torch().empty(b.value, dtype=_torch().uint8, device=self.device)

    def dgraph(self, g):
        """Padded-CSR device graph of a host CSR (off = row_ptr, len = row
        lengths); degrees are filled by step_contract."""
        torch = _torch()
        rp = np.ascontiguousarray(g.row_ptr, np.int64)
        d = DeviceGraph(int(g.n), max(int(rp[-1]), 1), self.device)
        d.off.copy_(torch.as_tensor(rp[:-1].astype(np.int32)))
        d.len.copy_(torch.as_tensor(np.diff(rp).astype(np.int32)))
        if rp[-1] > 0:
            d.col[:rp[-1]].copy_(torch.as_tensor(np.ascontiguousarray(g.col, np.int32)))
            d.w[:rp[-1]].copy_(torch.as_tensor(np.ascontiguousarray(g.w, np.int64)))
        return d

    def step_contract(self, src, labels=None, n2=None):
        n2 = src.n if labels is None else int(n2)
        dst = DeviceGraph(n2, src.cap, self.device)
        ws = self.step_workspace(src.n, src.cap)
        dmin, darg = ctypes.c_int64(), ctypes.c_int32()
        _check(lib().mc_step_contract(self.h, ctypes.byref(src.c()), _ptr(labels), n2, ctypes.byref(dst.c()),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(dmin),
                                      ctypes.byref(darg)))
        return dst, dmin.value, darg.value

    def step_components(self, n, a, b):
        torch = _torch()
        a = torch.as_tensor(np.ascontiguousarray(a, np.int32)).to(self.device)
        b = torch.as_tensor(np.ascontiguousarray(b, np.int32)).to(self.device)
        lab = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        n2 = ctypes.c_int32()
        ws = self.step_workspace(n, 1)
        _check(lib().mc_step_components(self.h, n, a.numel(), _ptr(a), _ptr(b), _ptr(lab), ctypes.byref(n2),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return lab[:n].cpu().numpy(), n2.value

    def step_pr12(self, g, lam):
        torch = _torch()
        flag = torch.zeros(g.cap, dtype=torch.uint8, device=self.device)
        ptr = torch.empty(g.n, dtype=torch.int32, device=self.device)
        lab = torch.empty(g.n, dtype=torch.int32, device=self.device)
        n2 = ctypes.c_int32()
        ws = self.step_workspace(g.n, g.cap)
        _check(lib().mc_step_pr12(self.h, ctypes.byref(g.c()), lam, _ptr(flag), _ptr(ptr), _ptr(lab),
                                  ctypes.byref(n2), ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return flag, ptr.cpu().numpy(), lab.cpu().numpy(), n2.value

    def step_pr34(self, g, lam, D, ptr2):
        """Reduction tests 3 and 4 (see mc_step_pr34): (flag4 per entry as a
        device tensor, accepted test-3 partner per vertex, labels, n2)."""
        torch = _torch()
        p = torch.as_tensor(np.ascontiguousarray(ptr2, np.int32)).to(self.device)
        flag = torch.zeros(g.cap, dtype=torch.uint8, device=self.device)
        acc = torch.empty(max(g.n, 1), dtype=torch.int32, device=self.device)
        lab = torch.empty(max(g.n, 1), dtype=torch.int32, device=self.device)
        n2 = ctypes.c_int32()
        ws = self.step_workspace(g.n, g.cap)
        _check(lib().mc_step_pr34(self.h, ctypes.byref(g.c()), lam, D, _ptr(p), _ptr(flag), _ptr(acc), _ptr(lab),
                                  ctypes.byref(n2), ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return flag, acc[:g.n].cpu().numpy(), lab[:g.n].cpu().numpy(), n2.value

    def step_lp(self, g, lab_in):
        """One label-propagation round on device graph g (see mc_step_lp);
        lab_in None: singleton labels (g must be normal)."""
        torch = _torch()
        a = None if lab_in is None else torch.as_tensor(np.ascontiguousarray(lab_in, np.int32)).to(self.device)
        out = torch.empty(max(g.n, 1), dtype=torch.int32, device=self.device)
        ws = self.step_workspace(g.n, g.cap)
        _check(lib().mc_step_lp(self.h, ctypes.byref(g.c()), None if a is None else _ptr(a), _ptr(out),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return out[:g.n].cpu().numpy()

    def step_capforest(self, g, lam, start=0, mode=CF_SEQUENTIAL, passes=1, shared=False, len_cap=0):
        """One CAPFOREST launch in the given mode (CF_SHARED, CF_SEQUENTIAL,
        CF_PRIVATE, CF_LEVELS); see mc_step_capforest."""
        torch = _torch()
        lab = torch.empty(g.n, dtype=torch.int32, device=self.device)
        order = torch.full((max(g.n, 4096),), -1, dtype=torch.int32, device=self.device)
        n2, ns, bl = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ba, lo = ctypes.c_int64(), ctypes.c_int64()
        ws = self.step_workspace(g.n, g.cap, passes)
        _check(lib().mc_step_capforest(self.h, ctypes.byref(g.c()), lam, start, int(mode), passes, int(shared),
                                       len_cap, _ptr(lab), ctypes.byref(n2), _ptr(order), ctypes.byref(ns),
                                       ctypes.byref(ba), ctypes.byref(bl), ctypes.byref(lo),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return {"labels": lab.cpu().numpy(), "n2": n2.value, "order": order[:ns.value].cpu().numpy(),
                "best_alpha": ba.value, "best_len": bl.value, "lam": lo.value}


def check_graph(g, symmetric=False):
    """Host-side checks of a graph (mc_check_graph; no GPU needed): the
    status code, 0 for a valid graph."""
    rp = np.ascontiguousarray(g.row_ptr, np.int32)
    col = np.ascontiguousarray(g.col, np.int32)
    w = np.ascontiguousarray(g.w, np.int64)
    nnz = int(getattr(g, "nnz", rp[-1] if rp.size else 0))
    csr = CSR(int(g.n), nnz, rp.ctypes.data if rp.size else 0, col.ctypes.data if col.size else 0,
              w.ctypes.data if w.size else 0, MC_HOST)
    return int(lib().mc_check_graph(ctypes.byref(csr), 1 if symmetric else 0))


class Server:
    """Continuous-batching request server (mc_server_*) on a context."""

    def __init__(self, ctx, hbm_bytes, max_inflight=0, max_request_n=0, max_request_nnz=0, solo_min_n=0,
                 solo_slots=0, deadline_ms=0.0):
        self.ctx = ctx
        self.opts = ServerOpts(hbm_bytes, max_inflight, max_request_n, max_request_nnz, solo_min_n, solo_slots,
                               deadline_ms)
        h = ctypes.c_void_p()
        _check(lib().mc_server_create(ctx.h, ctypes.byref(self.opts), ctypes.byref(h)))
        self.h = h
        self.n = {}

    def close(self):
        if getattr(self, "h", None):
            lib().mc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def capacity(self):
        e, v, k, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(lib().mc_server_capacity(self.h, ctypes.byref(e), ctypes.byref(v), ctypes.byref(k), ctypes.byref(b)))
        return {"entries": e.value, "vertices": v.value, "graphs": k.value, "bytes": b.value}

    def submit(self, g):
        rp = np.ascontiguousarray(g.row_ptr, np.int32)
        col = np.ascontiguousarray(g.col, np.int32)
        w = np.ascontiguousarray(g.w, np.int64)
        nnz = int(rp[-1])
        csr = CSR(int(g.n), nnz, rp.ctypes.data, col.ctypes.data if nnz else 0, w.ctypes.data if nnz else 0, MC_HOST)
        t = ctypes.c_uint64()
        _check(lib().mc_server_submit(self.h, ctypes.byref(csr), ctypes.byref(t)))
        self.n[t.value] = int(g.n)
        return t.value

    def step(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mc_server_step(self.h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def state(self, ticket):
        st = ctypes.c_int32()
        _check(lib().mc_server_state(self.h, ticket, ctypes.byref(st)))
        return st.value

    def poll(self, ticket):
        """None while running, else (lambda, side, stats dict)."""
        if self.state(ticket) < 2:
            return None
        lam = ctypes.c_int64()
        side = np.zeros(self.n[ticket], np.uint8)
        st = ReqStats()
        rc = lib().mc_server_poll(self.h, ticket, ctypes.byref(lam), side.ctypes.data, ctypes.byref(st))
        if rc == -6:
            return None
        _check(rc)
        del self.n[ticket]
        return lam.value, side, st.as_dict()

    def cancel(self, ticket):
        _check(lib().mc_server_cancel(self.h, ticket))


class DeviceGraph:
    """Padded CSR in device memory (see mc_dgraph in include/mincut_steps.h)."""

    def __init__(self, n, cap, device):
        torch = _torch()
        self.n, self.cap = int(n), int(cap)
        self.off = torch.zeros(max(self.n, 1), dtype=torch.int32, device=device)
        self.len = torch.zeros(max(self.n, 1), dtype=torch.int32, device=device)
        self.deg = torch.zeros(max(self.n, 1), dtype=torch.int64, device=device)
        self.col = torch.zeros(max(self.cap, 1), dtype=torch.int32, device=device)
        self.w = torch.zeros(max(self.cap, 1), dtype=torch.int64, device=device)

    def c(self):
        return DGraphC(self.n, self.cap, self.off.data_ptr(), self.len.data_ptr(), self.col.data_ptr(),
                       self.w.data_ptr(), self.deg.data_ptr())

    def to_canonical(self):
        """Host (row_ptr, col, w, deg) with every row sorted by target."""
        off = self.off[:self.n].cpu().numpy().astype(np.int64)
        ln = self.len[:self.n].cpu().numpy().astype(np.int64)
        col = self.col.cpu().numpy()
        w = self.w.cpu().numpy()
        rp = np.zeros(self.n + 1, np.int64)
        rp[1:] = np.cumsum(ln)
        rows = np.repeat(np.arange(self.n, dtype=np.int64), ln)
        pos = np.repeat(off - rp[:-1], ln) + np.arange(int(rp[-1]), dtype=np.int64)
        c, ww = col[pos], w[pos]
        o = np.lexsort((c, rows))
        oc, ow = c[o].astype(np.int32), ww[o].astype(np.int64)
        return rp.astype(np.int32), oc, ow, self.deg[:self.n].cpu().numpy()


_default_ctx = None


def mincut(g, **kw):
    """lambda and one side of a minimum cut of host graph g, on cuda:0."""
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(0)
    return _default_ctx.mincut(g, **kw)
