"""Python side of the HIP library: a plan object holding the C plan handle and its device workspace,
with thin wrappers that pass torch tensors' device pointers and the current HIP stream.

torch is used for device memory and streams only; every arithmetic step runs in libmrmf.so.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib as L


def _stream(device=None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _need_gpu(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")


def _site_array(sites):
    arr = (L.mrmf_site * len(sites))()
    for i, s in enumerate(sites):
        kind, k = (s.kind, s.k) if hasattr(s, "kind") else s
        arr[i].kind, arr[i].k = int(kind), int(k)
    return arr


def _local_array(ops):
    """ctypes array of mrmf_local_op (and the value buffers it points into, to keep alive)."""
    arr = (L.mrmf_local_op * max(1, len(ops)))()
    keep = []
    for i, o in enumerate(ops):
        v = np.ascontiguousarray(np.asarray(o.values, dtype=np.float64))
        keep.append(v)
        arr[i].site, arr[i].shift = int(o.site), int(o.shift)
        arr[i].values = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return arr, keep


def _term_array(terms):
    arr = (L.mrmf_term * max(1, len(terms)))()
    for i, t in enumerate(terms):
        if hasattr(t, "site_a"):
            sa, oa, sb, ob, p, w = t.site_a, t.op_a, t.site_b, t.op_b, t.param, t.w
        else:
            sa, oa, sb, ob, p, w = t
        w = complex(w)
        arr[i].site_a, arr[i].op_a, arr[i].site_b, arr[i].op_b = int(sa), int(oa), int(sb), int(ob)
        arr[i].param, arr[i].w_re, arr[i].w_im = int(p), w.real, w.imag
    return arr


class Plan:
    """A Hamiltonian structure (sites + terms) compiled by mrmf_plan_create, with its tables uploaded
    to a device workspace.  Couplings theta are passed per call."""

    def __init__(self, sites: Sequence, terms: Sequence, n_params: int, require_hermitian: bool = True,
                 device: str | torch.device = "cuda", local_ops: Sequence = ()):
        self._handle = ctypes.c_void_p()
        sa, ta = _site_array(sites), _term_array(terms)
        flags = L.MRMF_REQUIRE_HERMITIAN if require_hermitian else 0
        la, keep = _local_array(local_ops)
        L.call("mrmf_plan_create_ex", len(sites), sa, len(terms), ta, int(n_params), flags, len(local_ops), la,
               ctypes.byref(self._handle))
        del keep
        self._sites, self._terms = list(sites), list(terms)
        self._local = [(int(o.site), int(o.shift)) for o in local_ops]
        self.n_params = int(n_params)
        self.device = torch.device(device)
        D = ctypes.c_int64()
        L.call("mrmf_plan_dim", self._handle, ctypes.byref(D))
        self.D = int(D.value)
        n = ctypes.c_int32()
        L.call("mrmf_plan_n_offdiag", self._handle, ctypes.byref(n))
        self.n_offdiag = int(n.value)
        nb = ctypes.c_size_t()
        L.call("mrmf_plan_workspace_bytes", self._handle, ctypes.byref(nb))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        L.call("mrmf_plan_upload", self._handle, _ptr(self.ws), nb.value, _stream(self.device))
        torch.cuda.current_stream(self.device).synchronize()

    @classmethod
    def from_model(cls, model, **kw) -> "Plan":
        return cls(model.sites, model.terms, model.n_params, local_ops=getattr(model, "local_ops", ()), **kw)

    @property
    def handle(self):
        return self._handle

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            try:
                L.lib().mrmf_plan_destroy(h)
            except Exception:
                pass
            self._handle = None

    # ------------------------------------------------------------------ host queries
    def offsets(self):
        out = (ctypes.c_int64 * max(1, self.n_offdiag))()
        L.call("mrmf_plan_offsets", self._handle, out)
        return [int(out[i]) for i in range(self.n_offdiag)]

    def offdiag_terms(self):
        out = (ctypes.c_int32 * max(1, self.n_offdiag))()
        L.call("mrmf_plan_offdiag_terms", self._handle, out)
        return [int(out[i]) for i in range(self.n_offdiag)]

    # ------------------------------------------------------------------ device calls
    def theta(self, values, dtype=torch.float64) -> torch.Tensor:
        return torch.as_tensor(values, dtype=dtype).to(self.device)

    def matvec(self, theta: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """y = H(theta) x; complex128 -> mrmf_matvec_z, complex64 -> mrmf_matvec_c."""
        _need_gpu(x, "x")
        if x.numel() != self.D:
            raise ValueError(f"x has {x.numel()} entries, the basis has {self.D}")
        y = torch.empty_like(x) if out is None else out
        _need_gpu(y, "out", x.dtype)
        if x.dtype == torch.complex128:
            _need_gpu(theta, "theta", torch.float64)
            L.call("mrmf_matvec_z", self._handle, _ptr(self.ws), _ptr(theta), _ptr(x), _ptr(y),
                   _stream(self.device))
        elif x.dtype == torch.complex64:
            _need_gpu(theta, "theta", torch.float32)
            L.call("mrmf_matvec_c", self._handle, _ptr(self.ws), _ptr(theta), _ptr(x), _ptr(y),
                   _stream(self.device))
        else:
            raise ValueError("x must be complex128 or complex64")
        return y

    def debug_sources(self, F0: int, count: int) -> torch.Tensor:
        out = torch.empty((count, self.n_offdiag), dtype=torch.int64, device=self.device)
        L.call("mrmf_debug_sources", self._handle, _ptr(self.ws), int(F0), int(count), _ptr(out),
               _stream(self.device))
        return out

    # ------------------------------------------------------------------ adjoint
    def adjoint(self, theta: torch.Tensor, x: torch.Tensor, g: torch.Tensor):
        """(grad_x, grad_theta) of y = H(theta) x for the upstream gradient g (mrmf_adjoint_z):
        grad_x = H g (H Hermitian), grad_theta[p] = Re <g|h_p x>.  c128 / float64 only."""
        _need_gpu(theta, "theta", torch.float64)
        _need_gpu(x, "x", torch.complex128)
        _need_gpu(g, "g", torch.complex128)
        if x.numel() != self.D or g.numel() != self.D:
            raise ValueError("x and g must have D entries")
        gx = torch.empty_like(g)
        gt = torch.empty(max(1, self.n_params), dtype=torch.float64, device=self.device)
        nb = ctypes.c_size_t()
        L.call("mrmf_adjoint_scratch_bytes", self._handle, ctypes.byref(nb))
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        L.call("mrmf_adjoint_z", self._handle, _ptr(self.ws), _ptr(theta), _ptr(x), _ptr(g), _ptr(gx),
               _ptr(gt), _ptr(scratch), nb.value, _stream(self.device))
        return gx, gt[: self.n_params]

    # ------------------------------------------------------------------ time propagation
    def norm_bound(self, theta) -> float:
        """Upper bound on ||H(theta)||_2 (mrmf_plan_norm_bound; theta on the host or the device)."""
        th = np.ascontiguousarray(theta.detach().cpu().numpy() if isinstance(theta, torch.Tensor) else theta,
                                  dtype=np.float64)
        if th.size < self.n_params:
            raise ValueError("theta has fewer than n_params entries")
        out = ctypes.c_double()
        L.call("mrmf_plan_norm_bound", self._handle, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
               ctypes.byref(out))
        return float(out.value)

    def spectral_bounds(self, theta: torch.Tensor) -> tuple:
        """(e_min, e_max) containing the spectrum of H(theta), from the Gershgorin discs of its rows
        (mrmf_spectral_bounds, one device pass over the rows).  theta: float64 [n_params] on the device, or
        [S, n_params] for the ends over S coupling vectors (mrmf_spectral_bounds_many: one pass for all of
        them; one pass per vector for plans that form does not take)."""
        return _spectral_bounds("mrmf_spectral_bounds", self._handle, self.ws, self.n_params, self.device, theta)

    def propagate(self, theta: torch.Tensor, x0: torch.Tensor, dt: float, n_steps: int = 1,
                  bounds: tuple | str | None = None, tol: float = 1e-12, out: torch.Tensor | None = None) -> dict:
        """x = exp(-i H dt)^n_steps x0 by Chebyshev expansion (mrmf_propagate_z).  theta: float64
        [n_params] (fixed H) or [n_steps, n_params] (a piecewise-constant drive, row s for step s).
        bounds = (e_min, e_max) must contain the spectrum of every step's H; default (None): the extreme
        Gershgorin ends over the steps' distinct theta rows (spectral_bounds), widened by a relative
        1e-9 against rounding; "norm": +-max over the steps of mrmf_plan_norm_bound (looser, host only).
        Returns dict(x=..., n_terms=Chebyshev terms over the whole call, bounds); with a fixed H the steps
        are taken as one longer step where the series stays short (set_tuning(cheb_merge=0): one series per
        step)."""
        _need_gpu(x0, "x0", torch.complex128)
        if x0.numel() != self.D:
            raise ValueError("x0 has the wrong length")
        stride, bounds = self._propagation_args(theta, n_steps, bounds)
        x = torch.empty_like(x0) if out is None else out
        _need_gpu(x, "out", torch.complex128)
        nb = ctypes.c_size_t()
        L.call("mrmf_propagate_scratch_bytes", self._handle, ctypes.byref(nb))
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        nt = ctypes.c_int32()
        L.call("mrmf_propagate_z", self._handle, _ptr(self.ws), _ptr(theta), int(stride), float(dt), int(n_steps),
               float(bounds[0]), float(bounds[1]), float(tol), _ptr(x0), _ptr(x), _ptr(scratch), nb.value,
               ctypes.byref(nt), _stream(self.device))
        return dict(x=x, n_terms=int(nt.value), bounds=tuple(bounds), scratch=scratch)

    def _propagation_args(self, theta: torch.Tensor, n_steps: int, bounds, owner=None) -> tuple:
        """(theta_stride, (e_min, e_max)) of a propagation call: the stride from theta's shape and the
        bounds as described in propagate(); the default (Gershgorin) bounds are those of `owner` (this plan,
        or a sector of it), cached per coupling vector on the owner."""
        owner = self if owner is None else owner
        _need_gpu(theta, "theta", torch.float64)
        stride = 0
        if theta.dim() == 2:
            if theta.shape[0] < n_steps or theta.shape[1] != self.n_params:
                raise ValueError("theta must be [n_steps, n_params]")
            stride = self.n_params
        if bounds is None or isinstance(bounds, str):
            th = theta.detach().cpu().numpy().reshape(-1, max(1, self.n_params)) if self.n_params else np.zeros((1, 0))
            th = th[: max(1, n_steps)]
            if bounds == "norm":
                b = max(self.norm_bound(r) for r in th)
                b = b if b > 0 else 1.0
                bounds = (-b, b)
            elif bounds is None:
                # the distinct coupling vectors of the call, all in one device pass; cached on the owner
                # (a plan or a sector: its terms never change) by those vectors
                rows = np.ascontiguousarray(np.unique(th, axis=0) if th.shape[1] else th[:1])
                cache = owner.__dict__.setdefault("_gersh_cache", {})
                key = (rows.shape, rows.tobytes())
                if key not in cache:
                    if len(cache) >= 256:
                        cache.clear()
                    t = torch.from_numpy(rows).to(self.device)
                    cache[key] = owner.spectral_bounds(t if rows.shape[0] > 1 else t[0])
                lo, hi = cache[key]
                pad = 1e-9 * max(hi - lo, abs(lo), abs(hi), 1e-3)
                bounds = (lo - pad, hi + pad)
            else:
                raise ValueError(f"unknown bounds {bounds!r}")
        return stride, tuple(bounds)

    # ------------------------------------------------------------------ Lanczos
    def lanczos(self, theta: torch.Tensor, v0: torch.Tensor, m: int, precision: str = "z",
                reorth: str = "cgs2", theta_c: torch.Tensor | None = None, keep_basis: bool = False) -> dict:
        """Lowest eigenpair by device-resident Lanczos (mrmf_lanczos).  precision "z" (c128 matvec) or
        "c_in_z" (c64 matvec inside the FP64 recurrence); reorth "cgs2" (two Gram-Schmidt passes),
        "cgs2_cond" (the second only when the first shrank ||w|| by more than 1/sqrt(2)), "partial" (one
        pass only where Simon's estimate of the loss of orthogonality passes sqrt(eps), and the step after)
        or "none".  Returns device tensors alpha, beta, the Ritz vector u, result = [theta, residual
        estimate, explicit residual, steps] and counts = [second passes (cgs2_cond), passes (partial)]."""
        return _lanczos("mrmf_lanczos", self._handle, self.ws, self.D, self.device, theta, v0, m, precision,
                        reorth, theta_c, keep_basis)

    # ------------------------------------------------------------------ kernel selection
    KERNELS = {"auto": 0, "generic": 1, "specialized": 2}

    def set_kernel(self, kind: str = "auto", inner_sites: int = 0, unrolled_sites: int = -1):
        """Choose the matvec kernel: "generic", "specialized" (plan-specific, compiled on first use) or
        "auto"; inner_sites = 0 / unrolled_sites = -1 let the library pick the tiling."""
        L.call("mrmf_plan_set_kernel", self._handle, self.KERNELS[kind], int(inner_sites), int(unrolled_sites))

    TUNING = {"schedule": 0, "branch_skip": 1, "load_group": 2, "blocks_per_cu": 3, "variant": 4, "addressing": 5,
              "cheb_fused": 6, "waves_per_eu": 7, "far_loads": 8, "grad_blocks_per_cu": 9,
              "outer_first": 10, "unroll_top": 11, "far_dir": 12, "cheb_merge": 13}

    def set_tuning(self, **knobs):
        """Tuning knobs of the specialized kernel: schedule (0 windows, 1 per-XCD chunks, 2 block runs),
        branch_skip (0/1), load_group (channels issued ahead, 0 = default), blocks_per_cu (0 = as many as
        fit), variant (0 masked, 1 list), addressing (0 = 64-bit only where 32-bit offsets cannot reach,
        1 = always 64-bit), cheb_fused (1 = propagate with the fused Chebyshev-step kernel, 0 = matvec +
        update), waves_per_eu (0 = compiler's choice, else a minimum of resident waves per SIMD),
        far_loads (0 = default cache policy, k = gathers reaching 2^k bytes or more are non-temporal),
        far_dir (which of those: 0 both directions, 1 sources behind the row, 2 ahead), grad_blocks_per_cu (blocks per CU of the adjoint's generated coupling-gradient
        kernel, 0 = default), outer_first (k = the k most significant sites vary fastest in the sweep
        over super-tiles, 0 = index order), unroll_top (k = sites 0..k-1 join the unrolled copies, so terms
        between them and the low sites read LDS; 0 = off), cheb_merge (1 = propagate takes consecutive
        steps of a fixed H as one longer step, 0 = one Chebyshev series per step)."""
        for k, v in knobs.items():
            L.call("mrmf_plan_set_tuning", self._handle, self.TUNING[k], int(v))

    def autotune(self, theta: torch.Tensor, x: torch.Tensor, y: torch.Tensor | None = None,
                 use_cache: bool = True, kernel: str = "matvec") -> dict:
        """Pick the specialized kernel's shape for this plan and element type (x.dtype): from the tuning
        cache when the structure was tuned before, else by timing every candidate on these buffers
        (mrmf_plan_autotune) and recording the winner.  kernel="cheb" tunes the Chebyshev-step kernel of
        propagate (c128; y then needs 2 D elements)."""
        from . import tuning
        dt = L.MRMF_DTYPE_Z if x.dtype == torch.complex128 else L.MRMF_DTYPE_C
        if kernel == "cheb":
            if x.dtype != torch.complex128:
                raise ValueError("the Chebyshev-step kernel is c128")
            dt = L.MRMF_SOURCE_CHEB
            if y is None:
                y = torch.empty(2 * self.D, dtype=torch.complex128, device=x.device)
            if y.numel() < 2 * self.D:
                raise ValueError("y must hold 2 D elements for the Chebyshev-step kernel")
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        key = tuning.signature(self._sites, self._terms, dt, arch, self._local)
        ent = tuning.lookup(key) if use_cache else None
        if ent is None:
            y = torch.empty_like(x) if y is None else y
            _need_gpu(x, "x")
            _need_gpu(y, "y", x.dtype)
            out = (ctypes.c_int32 * 6)()
            st = L.lib().mrmf_plan_autotune(self._handle, dt, _ptr(self.ws), _ptr(theta), _ptr(x), _ptr(y),
                                           _stream(self.device), out)
            if st == L.MRMF_E_UNSUPPORTED:   # no specialized shape fits this plan: keep the default
                if dt != L.MRMF_SOURCE_CHEB:
                    self.prepare(x.dtype)
                return dict(kind="default", key=key)
            L.check(st, "mrmf_plan_autotune")
            ent = dict(variant=out[0], inner_sites=out[1], unrolled_sites=out[2], load_group=out[3],
                       us_per_call=out[4], D=self.D, unroll_top=out[5])
            if use_cache:
                tuning.store(key, ent)
        L.call("mrmf_plan_set_shape", self._handle, dt, int(ent["variant"]), int(ent["inner_sites"]),
               int(ent["unrolled_sites"]), int(ent["load_group"]), int(ent.get("unroll_top", 0)))
        if dt != L.MRMF_SOURCE_CHEB:
            self.prepare(x.dtype)
        return dict(ent, key=key)

    def prepare(self, dtype=torch.complex128):
        """Compile and load the kernel matvec will use for this element type (synchronous)."""
        dt = L.MRMF_DTYPE_Z if dtype == torch.complex128 else L.MRMF_DTYPE_C
        L.call("mrmf_plan_prepare", self._handle, dt)

    def grad_kernel_ready(self) -> bool:
        """Build the adjoint's generated coupling-gradient kernel now; False when the plan does not qualify
        for it (mrmf_adjoint_z then runs its generic pass)."""
        st = L.lib().mrmf_plan_prepare(self._handle, L.MRMF_SOURCE_GRAD)
        if st not in (0, L.MRMF_E_UNSUPPORTED):
            L.check(st, "mrmf_plan_prepare")
        return st == 0

    def kernel_info(self, dtype=torch.complex128) -> dict:
        dt = L.MRMF_DTYPE_Z if dtype == torch.complex128 else L.MRMF_DTYPE_C
        out = (ctypes.c_int32 * 8)()
        L.call("mrmf_plan_kernel_info", self._handle, dt, out)
        kind = {0: "auto", 1: "generic", 2: "specialized"}[out[0]]
        return dict(kind=kind, inner_sites=out[1], rows_per_block=out[2], block=out[3], grid=out[4],
                    super_tiles=out[5], unrolled_sites=out[6], copies=out[7])

    def kernel_source(self, dtype=torch.complex128) -> str:
        dt = L.MRMF_DTYPE_Z if dtype == torch.complex128 else L.MRMF_DTYPE_C
        n = ctypes.c_size_t()
        L.call("mrmf_plan_kernel_source", self._handle, dt, None, 0, ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value + 1)
        L.call("mrmf_plan_kernel_source", self._handle, dt, buf, n.value + 1, ctypes.byref(n))
        return buf.value.decode()


class MatvecFn(torch.autograd.Function):
    """y = H(theta) x with a hand-written backward: grad_x = H g (Hermitian H) and
    grad_theta[p] = Re <g|h_p x>, both from one mrmf_adjoint_z call.  Usage:
    ``MatvecFn.apply(plan, theta, x)`` with theta float64 and x complex128 on the GPU."""

    @staticmethod
    def forward(ctx, plan: Plan, theta: torch.Tensor, x: torch.Tensor):
        ctx.plan = plan
        ctx.save_for_backward(theta, x)
        return plan.matvec(theta.detach().contiguous(), x.detach().contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        theta, x = ctx.saved_tensors
        gx, gt = ctx.plan.adjoint(theta.detach().contiguous(), x.detach().contiguous(), g.contiguous())
        return None, (gt if ctx.needs_input_grad[1] else None), (gx if ctx.needs_input_grad[2] else None)


class Batch:
    """Many lattices applied to blocks of nvec c64 vectors in one persistent launch
    (mrmf_batch_matvec_c).  X and Y are flat complex64 tensors of total_elems entries; lattice b's
    block [D_b, nvec] starts at offsets[b].  theta_all is float32, the parameters of lattice 0, then
    lattice 1, ... (theta_offsets)."""

    def __init__(self, plans: Sequence[Plan], nvec: int = 8):
        self.plans = list(plans)          # the batch keeps pointers into its plans' host data
        self.nvec = int(nvec)
        self.device = self.plans[0].device
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        self._handle = ctypes.c_void_p()
        L.call("mrmf_batch_create", len(self.plans), arr, self.nvec, ctypes.byref(self._handle))
        n = len(self.plans)
        te = ctypes.c_int64()
        L.call("mrmf_batch_total_elems", self._handle, ctypes.byref(te))
        self.total_elems = int(te.value)
        offs = (ctypes.c_int64 * n)()
        L.call("mrmf_batch_offsets", self._handle, offs)
        self.offsets = [int(v) for v in offs]
        tho = (ctypes.c_int32 * (n + 1))()
        L.call("mrmf_batch_theta_offsets", self._handle, tho)
        self.theta_offsets = [int(v) for v in tho]
        nb = ctypes.c_size_t()
        L.call("mrmf_batch_workspace_bytes", self._handle, ctypes.byref(nb))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        L.call("mrmf_batch_upload", self._handle, _ptr(self.ws), nb.value, _stream(self.device))
        torch.cuda.current_stream(self.device).synchronize()

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            try:
                L.lib().mrmf_batch_destroy(h)
            except Exception:
                pass
            self._handle = None

    def block(self, T: torch.Tensor, b: int) -> torch.Tensor:
        """View of lattice b's [D_b, nvec] block inside a flat batch tensor."""
        D = self.plans[b].D
        return T[self.offsets[b]: self.offsets[b] + D * self.nvec].view(D, self.nvec)

    shared_input = False

    def share_input(self, on: bool = True):
        """Every lattice reads the one input block at the start of X (mrmf_batch_share_input): a parameter
        sweep applies its couplings to the same vectors without a copy per lattice.  X then needs
        input_elems entries."""
        L.call("mrmf_batch_share_input", self._handle, 1 if on else 0)
        self.shared_input = bool(on)

    @property
    def input_elems(self) -> int:
        """Entries X needs: total_elems, or one padded block with a shared input."""
        if not self.shared_input:
            return self.total_elems
        return (self.plans[0].D * self.nvec + 31) // 32 * 32

    def _check(self, theta_all, X, Y):
        _need_gpu(theta_all, "theta_all", torch.float32)
        _need_gpu(X, "X", torch.complex64)
        _need_gpu(Y, "Y", torch.complex64)
        if X.numel() < self.input_elems or Y.numel() < self.total_elems:
            raise ValueError("X needs input_elems entries and Y total_elems")
        if theta_all.numel() < self.theta_offsets[-1]:
            raise ValueError("theta_all is too short")

    def matvec(self, theta_all: torch.Tensor, X: torch.Tensor, Y: torch.Tensor | None = None) -> torch.Tensor:
        if Y is None:
            Y = torch.empty(self.total_elems, dtype=torch.complex64, device=X.device)
        self._check(theta_all, X, Y)
        L.call("mrmf_batch_matvec_c", self._handle, _ptr(self.ws), _ptr(theta_all), _ptr(X), _ptr(Y),
               _stream(self.device))
        return Y

    def capture(self, theta_all: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, stream: torch.cuda.Stream):
        """Capture the launch for these buffers into a hipGraph owned by the batch (on a non-default
        stream); replay() launches it."""
        self._check(theta_all, X, Y)
        L.call("mrmf_batch_graph_capture", self._handle, _ptr(self.ws), _ptr(theta_all), _ptr(X), _ptr(Y),
               ctypes.c_void_p(stream.cuda_stream))

    def replay(self, stream: torch.cuda.Stream | None = None):
        s = stream.cuda_stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        L.call("mrmf_batch_graph_launch", self._handle, ctypes.c_void_p(s))

    def autotune(self, theta_all: torch.Tensor, X: torch.Tensor, Y: torch.Tensor) -> dict:
        """Time every candidate launch shape on these buffers and keep the fastest."""
        self._check(theta_all, X, Y)
        out = (ctypes.c_int32 * 3)()
        L.call("mrmf_batch_autotune", self._handle, _ptr(self.ws), _ptr(theta_all), _ptr(X), _ptr(Y),
               _stream(self.device), out)
        return dict(self.shape(), candidate=out[2])

    def set_shape(self, tile_rows_max: int, block: int, schedule: str | None = None):
        """Launch shape: tiles of at most tile_rows_max rows ((64, 128, 256, 512) * 8 / nvec), block
        threads (a multiple of 64, at most 512 and 4096 / nvec) and, when given, the work schedule
        ("runs": a contiguous run of items per block; "windows": consecutive items side by side;
        "xcd_chunk": each XCD its own eighth of the items, its blocks side by side)."""
        L.call("mrmf_batch_set_shape", self._handle, int(tile_rows_max), int(block))
        if schedule is not None:
            L.call("mrmf_batch_set_schedule", self._handle,
                   {"runs": L.MRMF_BATCH_SCHED_RUNS, "windows": L.MRMF_BATCH_SCHED_WINDOWS,
                    "xcd_chunk": L.MRMF_BATCH_SCHED_XCD_CHUNK}[schedule])

    def shape(self) -> dict:
        out = (ctypes.c_int32 * 4)()
        L.call("mrmf_batch_get_shape", self._handle, out)
        return dict(tile_rows_max=out[0], block=out[1], schedule=("runs", "windows", "xcd_chunk")[out[2]],
                    grid=out[3])


def _spectral_bounds(fn: str, handle, ws, n_params: int, dev, theta: torch.Tensor) -> tuple:
    """Gershgorin ends through fn (mrmf_spectral_bounds or mrmf_sector_spectral_bounds) for one coupling
    vector, or through fn + "_many" for the rows of a [S, n_params] tensor (per row when the one-pass form
    does not take the plan)."""
    _need_gpu(theta, "theta", torch.float64)
    nb = ctypes.c_size_t()
    L.call(fn + "_scratch_bytes", handle, ctypes.byref(nb))
    scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    th = theta.contiguous()
    if th.dim() == 2:
        if th.shape[1] != n_params or th.shape[0] < 1:
            raise ValueError("theta must be [S, n_params] with S >= 1")
        st = getattr(L.lib(), fn + "_many")(handle, _ptr(ws), _ptr(th), n_params, th.shape[0], _ptr(out),
                                            _ptr(scratch), nb.value, _stream(dev))
        if st == L.MRMF_E_UNSUPPORTED:
            ends = [_spectral_bounds(fn, handle, ws, n_params, dev, r) for r in th]
            return min(e[0] for e in ends), max(e[1] for e in ends)
        L.check(st, fn + "_many")
    else:
        if th.numel() < n_params:
            raise ValueError("theta has fewer than n_params entries")
        L.call(fn, handle, _ptr(ws), _ptr(th), _ptr(out), _ptr(scratch), nb.value, _stream(dev))
    lo, hi = out.cpu().tolist()
    return lo, hi


def _lanczos(fn: str, handle, ws, D: int, dev, theta, v0, m, precision, reorth, theta_c, keep_basis) -> dict:
    """Shared marshalling of mrmf_lanczos / mrmf_sector_lanczos (same arguments, vectors of length D)."""
    _need_gpu(theta, "theta", torch.float64)
    _need_gpu(v0, "v0", torch.complex128)
    if v0.numel() != D:
        raise ValueError("v0 has the wrong length")
    prec = {"z": L.MRMF_PREC_Z, "c_in_z": L.MRMF_PREC_C_IN_Z}[precision]
    ro = {"cgs2": L.MRMF_REORTH_CGS2, "cgs2_cond": L.MRMF_REORTH_CGS2_COND, "partial": L.MRMF_REORTH_PARTIAL,
          "none": L.MRMF_REORTH_NONE}[reorth]
    if prec == L.MRMF_PREC_C_IN_Z:
        if theta_c is None:
            theta_c = theta.to(torch.float32)
        _need_gpu(theta_c, "theta_c", torch.float32)
    V = torch.empty((m + 1, D), dtype=torch.complex128, device=dev)
    alpha = torch.zeros(m, dtype=torch.float64, device=dev)
    beta = torch.zeros(m, dtype=torch.float64, device=dev)
    result = torch.full((4,), float("nan"), dtype=torch.float64, device=dev)
    u = torch.empty(D, dtype=torch.complex128, device=dev)
    nb = ctypes.c_size_t()
    L.call(fn + "_scratch_bytes", handle, int(m), prec, ctypes.byref(nb))
    scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    L.call(fn, handle, _ptr(ws), _ptr(theta), _ptr(theta_c) if theta_c is not None else None, prec, int(m), ro,
           _ptr(v0), _ptr(V), _ptr(alpha), _ptr(beta), _ptr(result), _ptr(u), _ptr(scratch), nb.value,
           _stream(dev))
    counts = torch.zeros(2, dtype=torch.int32, device=dev)
    L.call("mrmf_lanczos_counts", _ptr(scratch), _ptr(counts), _stream(dev))
    out = dict(alpha=alpha, beta=beta, result=result, u=u, scratch=scratch, counts=counts)
    if keep_basis:
        out["V"] = V
    return out


class Sweep:
    """A parameter sweep of one plan by linearity: H(theta) = sum_p theta_p h_p, so the products at K coupling
    vectors are Y_k = sum_p theta_kp (h_p X).  The P group products h_p X come from one batched launch of P
    copies of the plan with a shared input and unit coupling vectors (mrmf_batch_matvec_c), the K outputs
    from one combining pass (mrmf_sweep_combine_c).  X: nvec c64 vectors as one [D, nvec] block (input_elems
    entries); output k is block(Y, k)."""

    def __init__(self, plan: "Plan", nvec: int = 8):
        P = plan.n_params
        if not 1 <= P <= 16:
            raise ValueError("a sweep by linearity needs 1 to 16 couplings")
        self.plan, self.nvec, self.P, self.device = plan, int(nvec), P, plan.device
        self.basis = Batch([plan] * P, self.nvec)
        self.basis.share_input(True)
        self.n = plan.D * self.nvec
        self.stride = (self.n + 31) // 32 * 32          # the batch's block pitch (offsets padded to 32)
        if P > 1 and self.basis.offsets[1] - self.basis.offsets[0] != self.stride:
            raise RuntimeError("unexpected batch block pitch")
        self.input_elems = self.basis.input_elems
        self.unit = torch.eye(P, dtype=torch.float32, device=self.device).reshape(-1).contiguous()
        self.G = torch.empty(self.basis.total_elems, dtype=torch.complex64, device=self.device)

    def block(self, Y: torch.Tensor, k: int) -> torch.Tensor:
        """View of output k, [D, nvec]."""
        return Y[k * self.stride: k * self.stride + self.n].view(self.plan.D, self.nvec)

    def run(self, thetas: torch.Tensor, X: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """thetas: float32 [K, P] on the device; X: complex64, at least input_elems entries.  Returns Y with
        K blocks of stride entries."""
        _need_gpu(thetas, "thetas", torch.float32)
        if thetas.dim() != 2 or thetas.shape[1] != self.P:
            raise ValueError("thetas must be [K, n_params]")
        K = int(thetas.shape[0])
        Y = torch.empty(K * self.stride, dtype=torch.complex64, device=self.device) if out is None else out
        _need_gpu(Y, "out", torch.complex64)
        if Y.numel() < K * self.stride:
            raise ValueError("out needs K * stride entries")
        self.basis.matvec(self.unit, X, self.G)
        L.call("mrmf_sweep_combine_c", _ptr(thetas.contiguous()), K, self.P, self.n, _ptr(self.G), self.stride,
               _ptr(Y), self.stride, _stream(self.device))
        return Y


class Sector:
    """Restricted basis of the states whose local digits sum to digit_sum (mrmf_sector_*): packed vectors
    of length dim in ascending full-basis order, the matvec P H P^T, labels, lookup and Lanczos."""

    def __init__(self, plan: Plan, digit_sum: int):
        self.device = plan.device
        self.n_params = plan.n_params
        self.digit_sum = int(digit_sum)
        self._plan = plan   # spectral bounds for propagate()
        self._handle = ctypes.c_void_p()
        L.call("mrmf_sector_create", plan.handle, self.digit_sum, ctypes.byref(self._handle))
        n = ctypes.c_int64()
        L.call("mrmf_sector_dim", self._handle, ctypes.byref(n))
        self.dim = int(n.value)
        self.n_sites = len(plan._sites)
        nb = ctypes.c_size_t()
        L.call("mrmf_sector_workspace_bytes", self._handle, ctypes.byref(nb))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        L.call("mrmf_sector_upload", self._handle, _ptr(self.ws), nb.value, _stream(self.device))
        torch.cuda.current_stream(self.device).synchronize()

    @staticmethod
    def digit_sum_of(sites, magnetization: float) -> int:
        """Digit sum of the fixed-total-S_z sector M (spin sites only: n = m + s)."""
        q = magnetization + sum(0.5 * (s.k if hasattr(s, "k") else s[1]) for s in sites)
        if abs(q - round(q)) > 1e-9:
            raise ValueError("M + sum s_i must be an integer")
        return int(round(q))

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            try:
                L.lib().mrmf_sector_destroy(h)
            except Exception:
                pass
            self._handle = None

    def generated(self, dtype=torch.complex128) -> bool:
        """True when the matvec of this element type runs the kernel generated for the sector (built now
        if it was not yet), False when it runs the generic one."""
        used = ctypes.c_int32()
        L.call("mrmf_sector_generated", self._handle,
               L.MRMF_DTYPE_Z if dtype == torch.complex128 else L.MRMF_DTYPE_C, ctypes.byref(used))
        return bool(used.value)

    def matvec(self, theta: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """y = P H(theta) P^T x (c128 with float64 theta, or c64 with float32 theta)."""
        f32 = x.dtype == torch.complex64
        _need_gpu(x, "x", torch.complex64 if f32 else torch.complex128)
        _need_gpu(theta, "theta", torch.float32 if f32 else torch.float64)
        if x.numel() != self.dim:
            raise ValueError("x has the wrong length")
        y = torch.empty_like(x) if out is None else out
        _need_gpu(y, "out", x.dtype)
        L.call("mrmf_sector_matvec_c" if f32 else "mrmf_sector_matvec_z", self._handle, _ptr(self.ws), _ptr(theta),
               _ptr(x), _ptr(y), _stream(self.device))
        return y

    def labels(self, r0: int = 0, count: int | None = None) -> torch.Tensor:
        """Full-basis index of packed rows r0 .. r0 + count - 1 (int64 device tensor)."""
        count = self.dim - r0 if count is None else int(count)
        out = torch.empty(max(1, count), dtype=torch.int64, device=self.device)
        scratch = torch.empty(max(1, self.n_sites), dtype=torch.int64, device=self.device)
        L.call("mrmf_sector_labels", self._handle, _ptr(self.ws), int(r0), count, _ptr(out), _ptr(scratch),
               scratch.numel() * 8, _stream(self.device))
        return out[:count]

    def lookup(self, F: torch.Tensor) -> torch.Tensor:
        """Packed row of each full-basis index (int64 device tensor), -1 outside the sector."""
        _need_gpu(F, "F", torch.int64)
        out = torch.empty_like(F)
        L.call("mrmf_sector_lookup", self._handle, _ptr(self.ws), _ptr(F), F.numel(), _ptr(out),
               _stream(self.device))
        return out

    def lanczos(self, theta: torch.Tensor, v0: torch.Tensor, m: int, precision: str = "z",
                reorth: str = "cgs2", theta_c: torch.Tensor | None = None, keep_basis: bool = False) -> dict:
        """Lowest eigenpair in the sector (mrmf_sector_lanczos); the results of Plan.lanczos."""
        return _lanczos("mrmf_sector_lanczos", self._handle, self.ws, self.dim, self.device, theta, v0, m,
                        precision, reorth, theta_c, keep_basis)

    def spectral_bounds(self, theta: torch.Tensor) -> tuple:
        """(e_min, e_max) containing the spectrum of P H(theta) P^T, from the Gershgorin discs of the
        sector's rows (mrmf_sector_spectral_bounds).  theta: float64 [n_params] on the device, or
        [S, n_params] for the ends over S coupling vectors (mrmf_sector_spectral_bounds_many)."""
        return _spectral_bounds("mrmf_sector_spectral_bounds", self._handle, self.ws, self.n_params, self.device,
                                theta)

    def norm_bound(self, theta) -> float:
        """The plan's host norm bound (it bounds P H P^T as well)."""
        return self._plan.norm_bound(theta)

    def propagate(self, theta: torch.Tensor, x0: torch.Tensor, dt: float, n_steps: int = 1,
                  bounds: tuple | str | None = None, tol: float = 1e-12, out: torch.Tensor | None = None) -> dict:
        """x = exp(-i P H P^T dt)^n_steps x0 on packed sector vectors (mrmf_sector_propagate_z); theta,
        bounds and the result as in Plan.propagate, the default bounds from the sector's own Gershgorin
        discs (spectral_bounds; the plan's bounds contain the sector's spectrum as well, but less tightly)."""
        _need_gpu(x0, "x0", torch.complex128)
        if x0.numel() != self.dim:
            raise ValueError("x0 has the wrong length")
        stride, bounds = self._plan._propagation_args(theta, n_steps, bounds, owner=self)
        x = torch.empty_like(x0) if out is None else out
        _need_gpu(x, "out", torch.complex128)
        nb = ctypes.c_size_t()
        L.call("mrmf_sector_propagate_scratch_bytes", self._handle, ctypes.byref(nb))
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        nt = ctypes.c_int32()
        L.call("mrmf_sector_propagate_z", self._handle, _ptr(self.ws), _ptr(theta), int(stride), float(dt),
               int(n_steps), float(bounds[0]), float(bounds[1]), float(tol), _ptr(x0), _ptr(x), _ptr(scratch),
               nb.value, ctypes.byref(nt), _stream(self.device))
        return dict(x=x, n_terms=int(nt.value), bounds=tuple(bounds), scratch=scratch)
