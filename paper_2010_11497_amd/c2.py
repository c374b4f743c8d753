"""Python binding of libc2.so (include/c2.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory (tensors) and the stream (torch's
current stream).  If libc2.so is missing or fails to load, every call raises;
there is no fallback.

All array arguments are torch tensors on the GPU with the dtype and shape the
C declarations state; outputs are allocated here unless passed in.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libc2.so")

C2_OK = 0
C2_PAD = 0xFFFFFFFF
FORM_PLAIN = 0
FORM_BATCHED = 1
(OP_VALIDATE, OP_CLUSTER, OP_LOCAL_KNN, OP_BUILD, OP_BRUTE_FORCE, OP_FINGERPRINT,
 OP_LOCAL_KNN_ALG2, OP_LOCAL_KNN_MIN) = range(8)

# every entry point of include/c2.h
SYMBOLS = ["c2_last_error", "c2_workspace_bytes", "c2_validate", "c2_hash_items", "c2_frh_keys",
           "c2_cluster", "c2_cluster_keys", "c2_check_complete", "c2_local_knn",
           "c2_local_knn_alg2", "c2_merge", "c2_build", "c2_build_noalloc",
           "c2_brute_force", "c2_fingerprint", "c2_assign_hidden", "c2_assign_keys",
           "c2_embag", "c2_embag_backward", "c2_assign_train_workspace_bytes",
           "c2_assign_train_grad", "c2_adam_step", "c2_graph_create", "c2_graph_launch",
           "c2_graph_destroy"]
ASSIGN_DIM, ASSIGN_HIDDEN = 64, 256


class C2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("c2 status %d: %s" % (status, msg))
        self.status = status


class Profiles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint32), ("nnz", ctypes.c_uint64),
                ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("t", ctypes.c_uint32), ("b", ctypes.c_uint32), ("cap", ctypes.c_uint32),
                ("k", ctypes.c_uint32)]


class Hyrec(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_uint32), ("max_iter", ctypes.c_uint32),
                ("delta", ctypes.c_double), ("seed", ctypes.c_uint64)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("w_neg", ctypes.c_float), ("w_bal", ctypes.c_float), ("w_ent", ctypes.c_float)]


class Tuning(ctypes.Structure):
    _fields_ = [("mfma_min_rows", ctypes.c_uint32), ("persistent_wgs", ctypes.c_uint32),
                ("split_rounds", ctypes.c_uint32), ("group_tiles", ctypes.c_uint32),
                ("cluster_path", ctypes.c_uint32),
                ("ev_knn_begin", ctypes.c_void_p), ("ev_knn_end", ctypes.c_void_p),
                ("tile32_max", ctypes.c_uint32), ("tile64_max", ctypes.c_uint32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libc2.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError("libc2.so is not built (%s); run python -m "
                                "paper_2010_11497_amd.build" % path)
    L = ctypes.CDLL(path)
    P, u32, u64, i32, sz = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                            ctypes.c_size_t)
    PP, PA, PT = ctypes.POINTER(Profiles), ctypes.POINTER(Params), ctypes.POINTER(Tuning)
    L.c2_last_error.restype = ctypes.c_char_p
    L.c2_workspace_bytes.argtypes = [u32, u32, u64, PA, i32]
    L.c2_workspace_bytes.restype = sz
    L.c2_validate.argtypes = [PP, P, sz, P]
    L.c2_hash_items.argtypes = [P, u32, u32, u32, P, P]
    L.c2_frh_keys.argtypes = [PP, P, u32, P, P]
    L.c2_cluster.argtypes = [PP, P, PA, i32, PT, P, P, P, P, sz, P]
    L.c2_cluster_keys.argtypes = [PP, P, P, PA, i32, PT, P, P, P, P, sz, P]
    L.c2_check_complete.argtypes = [P, P]
    L.c2_local_knn.argtypes = [PP, P, P, P, PA, i32, PT, P, P, P, sz, P]
    L.c2_local_knn_alg2.argtypes = [PP, P, P, P, PA, ctypes.POINTER(Hyrec), PT, P, P, P, sz, P]
    L.c2_merge.argtypes = [PP, P, P, PA, P, P, P, P]
    L.c2_build.argtypes = [PP, P, PA, i32, PT, P, P, P, P, sz, P]
    L.c2_build_noalloc.argtypes = [PP, P, PA, i32, PT, P, P, P, P, P]
    L.c2_brute_force.argtypes = [PP, u32, P, P, P, P, sz, P]
    L.c2_fingerprint.argtypes = [PP, P, u32, P, P, ctypes.POINTER(u64), P, sz, P]
    L.c2_assign_hidden.argtypes = [PP, P, P, P, P, P]
    L.c2_assign_keys.argtypes = [P, u32, P, P, u32, u32, P, ctypes.c_float, P, P, P]
    L.c2_embag.argtypes = [PP, P, u32, P, P, P]
    L.c2_embag_backward.argtypes = [PP, P, u32, P, P, P]
    L.c2_assign_train_workspace_bytes.argtypes = [u32, u32, u32]
    L.c2_assign_train_workspace_bytes.restype = sz
    L.c2_assign_train_grad.argtypes = [PP, P, u32, P, P, P, P, P, u32, u32,
                                       ctypes.POINTER(TrainOpts), P, P, P, P, P, P, P, sz, P]
    f32 = ctypes.c_float
    L.c2_adam_step.argtypes = [P, P, P, P, u64, f32, f32, f32, f32, u32, P, P]
    L.c2_graph_create.argtypes = [PP, P, PA, PT, P, P, P, P, sz, P, ctypes.POINTER(P)]
    L.c2_graph_launch.argtypes = [P, P]
    L.c2_graph_destroy.argtypes = [P]
    for name in SYMBOLS:
        if name not in ("c2_last_error", "c2_workspace_bytes", "c2_assign_train_workspace_bytes"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def _check(st):
    if st != C2_OK:
        raise C2Error(st, load().c2_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _u32(shape, device):
    return torch.empty(shape, dtype=torch.int32, device=device)


class DeviceProfiles:
    """CSR profiles resident on the GPU (indptr int64[n+1], indices int32 view of
    uint32[nnz])."""

    def __init__(self, indptr, indices, n: int, m: int, device="cuda"):
        import numpy as np
        self.n, self.m = int(n), int(m)
        self.indptr = torch.as_tensor(np.asarray(indptr, dtype=np.int64)).to(device)
        self.indices = torch.as_tensor(np.asarray(indices, dtype=np.uint32).view(np.int32)).to(device)
        self.nnz = int(self.indices.numel())
        self.device = self.indptr.device
        self.c = Profiles(self.n, self.m, self.nnz, self.indptr.data_ptr(),
                          self.indices.data_ptr() if self.nnz else 0)

    @classmethod
    def from_synth(cls, P, device="cuda"):
        return cls(P.indptr, P.indices, P.n, P.m, device)

    @classmethod
    def from_device(cls, indptr: torch.Tensor, indices: torch.Tensor, n: int, m: int):
        """Wraps CSR tensors already on the GPU (indptr int64[n+1], indices
        int32[nnz]) without copying."""
        self = cls.__new__(cls)
        self.n, self.m = int(n), int(m)
        self.indptr, self.indices = indptr, indices
        self.nnz = int(indices.numel())
        self.device = indptr.device
        self.c = Profiles(self.n, self.m, self.nnz, indptr.data_ptr(),
                          indices.data_ptr() if self.nnz else 0)
        return self


def params(t, b, cap, k) -> Params:
    return Params(int(t), int(b), int(cap), int(k))


CLUSTER_AUTO, CLUSTER_GRID, CLUSTER_WORKGROUP = 0, 1, 2


def tuning(mfma_min_rows=0, persistent_wgs=0, split_rounds=0, group_tiles=0,
           cluster_path=CLUSTER_AUTO, events=None, tile32_max=0, tile64_max=0) -> Tuning:
    """Schedule and shape fields of c2_tuning (0 = the library's default;
    include/c2.h documents each); none changes a result.  events: optional
    (begin, end) torch.cuda.Event(enable_timing=True) pair recorded around the
    local-KNN kernel."""
    tu = Tuning(int(mfma_min_rows), int(persistent_wgs), int(split_rounds), int(group_tiles),
                int(cluster_path), None, None, int(tile32_max), int(tile64_max))
    if events is not None:
        for ev in events:
            ev.record()           # materialise the underlying hipEvent_t
        torch.cuda.current_stream().synchronize()
        tu.ev_knn_begin = ctypes.c_void_p(events[0].cuda_event)
        tu.ev_knn_end = ctypes.c_void_p(events[1].cuda_event)
    return tu


def workspace_bytes(P: DeviceProfiles, p: Optional[Params], op: int) -> int:
    L = load()
    nb = L.c2_workspace_bytes(P.n, P.m, P.nnz, ctypes.byref(p) if p is not None else None, op)
    if nb == 0:
        raise C2Error(-1, L.c2_last_error().decode())
    return int(nb)


def workspace(P: DeviceProfiles, p: Optional[Params], op: int) -> torch.Tensor:
    return torch.empty(workspace_bytes(P, p, op), dtype=torch.uint8, device=P.device)


C2_E_WORKSPACE = -3


def build_workspace(P: DeviceProfiles, tab: torch.Tensor, p: Params,
                    tune: Optional[Tuning] = None) -> torch.Tensor:
    """A c2_build workspace whose store holds this input's dictionary rows:
    the default size, grown by what one plain build reports as missing."""
    out = tuple(_u32((P.n, p.k), P.device) for _ in range(3))
    return _with_ws(lambda w: load().c2_build(ctypes.byref(P.c), _ptr(tab), ctypes.byref(p),
                                              FORM_PLAIN, ctypes.byref(tune) if tune else None,
                                              _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(w),
                                              w.numel(), _stream()),
                    None, lambda: workspace(P, p, OP_BUILD))


def store_need_bytes(ws: torch.Tensor) -> int:
    """Bytes of dictionary-row store the last local KNN on this workspace
    needed (the u64 at bytes 8..15 of its header, times 4)."""
    return 4 * int(ws[8:16].view(torch.int64).item())


def _with_ws(call, ws: Optional[torch.Tensor], default) -> torch.Tensor:
    """Runs call(ws).  When the workspace was allocated here (ws is None) and
    the partition's dictionary rows did not fit its store, allocates one
    larger by the store the library reports as needed and runs once more."""
    owned = ws is None
    ws = default() if owned else ws
    st = call(ws)
    if st == C2_E_WORKSPACE and owned:
        need = store_need_bytes(ws)
        if need > 0:
            ws = torch.empty(ws.numel() + need, dtype=torch.uint8, device=ws.device)
            st = call(ws)
    _check(st)
    return ws


def validate(P: DeviceProfiles, ws: Optional[torch.Tensor] = None) -> None:
    ws = workspace(P, None, OP_VALIDATE) if ws is None else ws
    _check(load().c2_validate(ctypes.byref(P.c), _ptr(ws), ws.numel(), _stream()))


def hash_items(tab: torch.Tensor, b: int, m: int, out=None) -> torch.Tensor:
    """tab: int64 view of uint64[t][4][256] on the GPU; returns int32 view of
    uint32[t][m]."""
    t = tab.shape[0]
    out = _u32((t, m), tab.device) if out is None else out
    _check(load().c2_hash_items(_ptr(tab), t, int(b), int(m), _ptr(out), _stream()))
    return out


def frh_keys(P: DeviceProfiles, bucket: torch.Tensor, out=None) -> torch.Tensor:
    t = bucket.shape[0]
    out = _u32((t, P.n), P.device) if out is None else out
    _check(load().c2_frh_keys(ctypes.byref(P.c), _ptr(bucket), t, _ptr(out), _stream()))
    return out


def cluster(P: DeviceProfiles, bucket: torch.Tensor, p: Params, form=FORM_PLAIN,
            tune: Optional[Tuning] = None, ws=None):
    """Returns (members int32[t*n], cl_off int32[t*n+1] (first ncl+1 valid),
    cl_cfg_off int32[t+1])."""
    NE = p.t * P.n
    members, cl_off, cfg = _u32(NE, P.device), _u32(NE + 1, P.device), _u32(p.t + 1, P.device)
    ws = workspace(P, p, OP_CLUSTER) if ws is None else ws
    _check(load().c2_cluster(ctypes.byref(P.c), _ptr(bucket), ctypes.byref(p), form,
                             ctypes.byref(tune) if tune else None, _ptr(members), _ptr(cl_off),
                             _ptr(cfg), _ptr(ws), ws.numel(), _stream()))
    return members, cl_off, cfg, ws


def cluster_keys(P: DeviceProfiles, keys: torch.Tensor, bucket: torch.Tensor, p: Params,
                 form=FORM_PLAIN, tune: Optional[Tuning] = None, ws=None):
    """Step 1 from per-user top-level keys (int32 view of uint32[t][n], < p.b),
    FastRandomHash on `bucket` splitting the clusters larger than p.cap.
    Returns as cluster()."""
    NE = p.t * P.n
    members, cl_off, cfg = _u32(NE, P.device), _u32(NE + 1, P.device), _u32(p.t + 1, P.device)
    ws = workspace(P, p, OP_CLUSTER) if ws is None else ws
    _check(load().c2_cluster_keys(ctypes.byref(P.c), _ptr(keys), _ptr(bucket), ctypes.byref(p),
                                  form, ctypes.byref(tune) if tune else None, _ptr(members),
                                  _ptr(cl_off), _ptr(cfg), _ptr(ws), ws.numel(), _stream()))
    return members, cl_off, cfg, ws


def check_complete(ws: torch.Tensor) -> None:
    _check(load().c2_check_complete(_ptr(ws), _stream()))


def local_knn(P: DeviceProfiles, members, cl_off, cl_cfg_off, p: Params, form=FORM_PLAIN,
              tune: Optional[Tuning] = None, ws=None, out=None):
    """Returns (part_id, part_I), int32 views of uint32[n][t][k]."""
    if out is None:
        out = (_u32((P.n, p.t, p.k), P.device), _u32((P.n, p.t, p.k), P.device))
    _with_ws(lambda w: load().c2_local_knn(ctypes.byref(P.c), _ptr(members), _ptr(cl_off),
                                           _ptr(cl_cfg_off), ctypes.byref(p), form,
                                           ctypes.byref(tune) if tune else None, _ptr(out[0]),
                                           _ptr(out[1]), _ptr(w), w.numel(), _stream()),
             ws, lambda: workspace(P, p, OP_LOCAL_KNN))
    return out


def local_knn_workspace(P: DeviceProfiles, members, cl_off, cl_cfg_off, p: Params,
                        tune: Optional[Tuning] = None) -> torch.Tensor:
    """A c2_local_knn workspace whose store holds this partition's dictionary
    rows: the default size, grown by what one plain run reports as missing."""
    out = (_u32((P.n, p.t, p.k), P.device), _u32((P.n, p.t, p.k), P.device))
    return _with_ws(lambda w: load().c2_local_knn(ctypes.byref(P.c), _ptr(members), _ptr(cl_off),
                                                  _ptr(cl_cfg_off), ctypes.byref(p), FORM_PLAIN,
                                                  ctypes.byref(tune) if tune else None,
                                                  _ptr(out[0]), _ptr(out[1]), _ptr(w), w.numel(),
                                                  _stream()),
                    None, lambda: workspace(P, p, OP_LOCAL_KNN))


def local_knn_alg2(P: DeviceProfiles, members, cl_off, cl_cfg_off, p: Params, rho=5,
                   max_iter=30, delta=0.001, seed=0, tune: Optional[Tuning] = None, ws=None,
                   out=None):
    """Algorithm 2: brute force below rho*k^2 members, deterministic Hyrec at or
    above (synchronous).  Returns (part_id, part_I) as local_knn()."""
    if out is None:
        out = (_u32((P.n, p.t, p.k), P.device), _u32((P.n, p.t, p.k), P.device))
    ws = workspace(P, p, OP_LOCAL_KNN_ALG2) if ws is None else ws
    hy = Hyrec(int(rho), int(max_iter), float(delta), int(seed))
    _check(load().c2_local_knn_alg2(ctypes.byref(P.c), _ptr(members), _ptr(cl_off),
                                    _ptr(cl_cfg_off), ctypes.byref(p), ctypes.byref(hy),
                                    ctypes.byref(tune) if tune else None, _ptr(out[0]),
                                    _ptr(out[1]), _ptr(ws), ws.numel(), _stream()))
    return out


def merge(P: DeviceProfiles, part_id, part_I, p: Params, out=None):
    """Returns (knn_id, knn_I, knn_U), int32 views of uint32[n][k]."""
    if out is None:
        out = tuple(_u32((P.n, p.k), P.device) for _ in range(3))
    _check(load().c2_merge(ctypes.byref(P.c), _ptr(part_id), _ptr(part_I), ctypes.byref(p),
                           _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream()))
    return out


def build(P: DeviceProfiles, tab: torch.Tensor, p: Params, form=FORM_PLAIN,
          tune: Optional[Tuning] = None, ws=None, out=None):
    if out is None:
        out = tuple(_u32((P.n, p.k), P.device) for _ in range(3))
    _with_ws(lambda w: load().c2_build(ctypes.byref(P.c), _ptr(tab), ctypes.byref(p), form,
                                       ctypes.byref(tune) if tune else None, _ptr(out[0]),
                                       _ptr(out[1]), _ptr(out[2]), _ptr(w), w.numel(), _stream()),
             ws, lambda: workspace(P, p, OP_BUILD))
    return out


def build_noalloc(P: DeviceProfiles, tab: torch.Tensor, p: Params, form=FORM_PLAIN,
                  tune: Optional[Tuning] = None, out=None, status=None):
    """c2_build on the library's fixed per-GPU workspace (no allocation in the
    call).  status: optional int32 tensor of one element that receives the
    split-completeness word (0 = complete)."""
    if out is None:
        out = tuple(_u32((P.n, p.k), P.device) for _ in range(3))
    _check(load().c2_build_noalloc(ctypes.byref(P.c), _ptr(tab), ctypes.byref(p), form,
                                   ctypes.byref(tune) if tune else None, _ptr(out[0]),
                                   _ptr(out[1]), _ptr(out[2]), _ptr(status), _stream()))
    return out


def fingerprint(P: DeviceProfiles, g: torch.Tensor, B: int, ws=None) -> DeviceProfiles:
    """GoldFinger fingerprints of the profiles as CSR profiles over B items
    (synchronous).  g: int32 view of uint32[m], positions < B, e.g.
    hash_items(tables, B, m)[0]."""
    L = load()
    indptr = torch.empty(P.n + 1, dtype=torch.int64, device=P.device)
    indices = _u32(max(P.nnz, 1), P.device)
    if ws is None:
        ws = workspace(P, params(1, B, 1, 1), OP_FINGERPRINT)
    nnz = ctypes.c_uint64()
    _check(L.c2_fingerprint(ctypes.byref(P.c), _ptr(g), int(B), _ptr(indptr), _ptr(indices),
                            ctypes.byref(nnz), _ptr(ws), ws.numel(), _stream()))
    return DeviceProfiles.from_device(indptr, indices[: nnz.value], P.n, B)


def build_goldfinger(P: DeviceProfiles, FP: DeviceProfiles, tab: torch.Tensor, p: Params,
                     tune: Optional[Tuning] = None):
    """C2 with GoldFinger local similarities (Section II-F): the clusters come
    from FastRandomHash on the profiles, the local KNN graphs and the merge
    from the fingerprints FP (see fingerprint()).  knn_I / knn_U are the
    fingerprints' intersection and union sizes."""
    bucket = hash_items(tab, p.b, P.m)
    members, cl_off, cfg, _ = cluster(P, bucket, p, FORM_PLAIN, tune)
    part = local_knn(FP, members, cl_off, cfg, p, FORM_PLAIN, tune)
    return merge(FP, part[0], part[1], p)


def assign_hidden(P: DeviceProfiles, E: torch.Tensor, W1: torch.Tensor, b1: torch.Tensor,
                  out=None) -> torch.Tensor:
    """h = ReLU(W1 mean(E[P_u]) + b1) for every user, bf16 [n][256].  E, W1
    bfloat16 tensors, b1 float32."""
    out = torch.empty((P.n, ASSIGN_HIDDEN), dtype=torch.bfloat16, device=P.device) \
        if out is None else out
    _check(load().c2_assign_hidden(ctypes.byref(P.c), _ptr(E), _ptr(W1), _ptr(b1), _ptr(out),
                                   _stream()))
    return out


def assign_keys(h: torch.Tensor, W2: torch.Tensor, b2: torch.Tensor, t: int, b: int,
                frh_keys: Optional[torch.Tensor] = None, min_gap: float = 0.0,
                with_gap: bool = False):
    """Per-head argmax of W2 h + b2: keys int32 view of uint32[t][n] (b + FRH
    key where the gap is below min_gap and frh_keys is given), and the gaps
    (float32 [t][n]) if with_gap."""
    n = h.shape[0]
    keys = _u32((t, n), h.device)
    gap = torch.empty((t, n), dtype=torch.float32, device=h.device) if with_gap else None
    _check(load().c2_assign_keys(_ptr(h), n, _ptr(W2), _ptr(b2), int(t), int(b),
                                 _ptr(frh_keys), float(min_gap), _ptr(keys), _ptr(gap),
                                 _stream()))
    return (keys, gap) if with_gap else keys


def embag(P: DeviceProfiles, E: torch.Tensor, rows: Optional[torch.Tensor] = None,
          nrows: Optional[int] = None) -> torch.Tensor:
    """fp32 mean of E rows over each listed user's items, [nrows][64]."""
    nrows = (rows.numel() if rows is not None else P.n) if nrows is None else nrows
    out = torch.empty((nrows, ASSIGN_DIM), dtype=torch.float32, device=P.device)
    _check(load().c2_embag(ctypes.byref(P.c), _ptr(rows), int(nrows), _ptr(E), _ptr(out),
                           _stream()))
    return out


def embag_backward(P: DeviceProfiles, grad: torch.Tensor, dE: torch.Tensor,
                   rows: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dE += gradient of embag() through grad (fp32, [nrows][64])."""
    _check(load().c2_embag_backward(ctypes.byref(P.c), _ptr(rows), int(grad.shape[0]),
                                    _ptr(grad), _ptr(dE), _stream()))
    return dE


def train_workspace(nrows: int, t: int, b: int, device="cuda") -> torch.Tensor:
    nb = load().c2_assign_train_workspace_bytes(int(nrows), int(t), int(b))
    if nb == 0:
        raise C2Error(C2_E_ARG, load().c2_last_error().decode())
    return torch.empty(nb, dtype=torch.uint8, device=device)


def assign_train_grad(P: DeviceProfiles, rows: torch.Tensor, E, W1, b1, W2, b2, t: int, b: int,
                      w_neg=1.0, w_bal=1.0, w_ent=1.0, ws=None, out=None):
    """One training step's loss parts (fp32 [5]: total, pair, non-neighbour,
    balance, entropy) and gradients (dE, dW1, db1, dW2, db2, fp32) for the
    batch rows (int32 view of u32 [2B]: users, then their neighbours).  E, W1,
    W2: the bf16 weights the forward reads; b1, b2 fp32."""
    R = int(rows.numel())
    dev = P.device
    if out is None:
        out = (torch.empty(5, dtype=torch.float32, device=dev),
               torch.empty((P.m, ASSIGN_DIM), dtype=torch.float32, device=dev),
               torch.empty((ASSIGN_HIDDEN, ASSIGN_DIM), dtype=torch.float32, device=dev),
               torch.empty(ASSIGN_HIDDEN, dtype=torch.float32, device=dev),
               torch.empty((t * b, ASSIGN_HIDDEN), dtype=torch.float32, device=dev),
               torch.empty(t * b, dtype=torch.float32, device=dev))
    ws = train_workspace(R, t, b, dev) if ws is None else ws
    o = TrainOpts(float(w_neg), float(w_bal), float(w_ent))
    loss, dE, dW1, db1, dW2, db2 = out
    _check(load().c2_assign_train_grad(ctypes.byref(P.c), _ptr(rows), R, _ptr(E), _ptr(W1),
                                       _ptr(b1), _ptr(W2), _ptr(b2), int(t), int(b),
                                       ctypes.byref(o), _ptr(loss), _ptr(dE), _ptr(dW1),
                                       _ptr(db1), _ptr(dW2), _ptr(db2), _ptr(ws), ws.numel(),
                                       _stream()))
    return out


def adam_step(param: torch.Tensor, grad: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor,
              lr: float, step: int, beta1=0.9, beta2=0.999, eps=1e-8,
              param_bf16: Optional[torch.Tensor] = None) -> None:
    """In-place Adam update of fp32 param (step counted from 1); param_bf16
    receives the updated values rounded to bf16."""
    _check(load().c2_adam_step(_ptr(param), _ptr(grad), _ptr(m1), _ptr(m2), param.numel(),
                               float(lr), float(beta1), float(beta2), float(eps), int(step),
                               _ptr(param_bf16), _stream()))


def build_from_buckets(P: DeviceProfiles, bucket: torch.Tensor, p: Params,
                       tune: Optional[Tuning] = None):
    """The three stages on an explicit bucket table (int32 view of
    uint32[t][m], values < p.b) instead of hashed items: clustering, local
    KNN and merge in the plain form.  With p.b = m and per-item permutation
    ranks as the table, and p.cap >= n, this is the MinHash clustering the
    paper compares FastRandomHash against (Section V-C, Table 4): one cluster
    per item that is some user's minimum, no splitting."""
    members, cl_off, cfg, _ = cluster(P, bucket, p, FORM_PLAIN, tune)
    part = local_knn(P, members, cl_off, cfg, p, FORM_PLAIN, tune)
    return merge(P, part[0], part[1], p)


def brute_force(P: DeviceProfiles, k: int, ws=None, out=None):
    if out is None:
        out = tuple(_u32((P.n, k), P.device) for _ in range(3))
    p = params(1, 1, 1, k)
    _with_ws(lambda w: load().c2_brute_force(ctypes.byref(P.c), int(k), _ptr(out[0]),
                                             _ptr(out[1]), _ptr(out[2]), _ptr(w), w.numel(),
                                             _stream()),
             ws, lambda: workspace(P, p, OP_BRUTE_FORCE))
    return out


class Graph:
    """The batched build captured as a HIP graph on fixed buffers."""

    def __init__(self, P: DeviceProfiles, tab: torch.Tensor, p: Params,
                 tune: Optional[Tuning] = None):
        self.P, self.tab, self.p = P, tab, p
        self.out = tuple(_u32((P.n, p.k), P.device) for _ in range(3))
        h = ctypes.c_void_p()
        # (creation runs one plain build first, which reports a store overflow)
        self.ws = _with_ws(lambda w: load().c2_graph_create(
            ctypes.byref(P.c), _ptr(tab), ctypes.byref(p), ctypes.byref(tune) if tune else None,
            _ptr(self.out[0]), _ptr(self.out[1]), _ptr(self.out[2]), _ptr(w), w.numel(),
            _stream(), ctypes.byref(h)), None, lambda: workspace(P, p, OP_BUILD))
        self.h = h

    def launch(self):
        _check(load().c2_graph_launch(self.h, _stream()))
        return self.out

    def check(self):
        check_complete(self.ws)

    def close(self):
        if self.h:
            load().c2_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_u32(t: torch.Tensor):
    """Copy a device int32 view back as a numpy uint32 array."""
    return t.cpu().numpy().view("uint32")


def tables_to_device(tab, device="cuda") -> torch.Tensor:
    import numpy as np
    return torch.as_tensor(np.ascontiguousarray(tab, dtype=np.uint64).view(np.int64)).to(device)
