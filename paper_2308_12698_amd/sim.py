"""Torch-facing binding of the C ABI: device tensors in, pointers out.

PyTorch supplies device memory and the current stream; every step of the
simulation runs in the HIP kernels of ``libpotato.so``.  Nothing here
computes any part of the method.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os
import re
import weakref

import torch

from . import _lib as L

N_ROWS = 30            # state rows per agent (include/potato.h)
N_CARRY = 10           # rounding-carry rows per agent
N_CKPT = 40            # rows of a checkpoint slot: the state, then its carries


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _state(state, carry):
    """potato_state of a [30, ld] state and an optional [10, carry_ld] carry."""
    return L.State(C.c_void_p(state.data_ptr()), state.stride(0),
                   None if carry is None else C.c_void_p(carry.data_ptr()),
                   0 if carry is None else carry.stride(0))


def _stream_handle(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check_rows(name, t, rows, n, dtype=torch.float32):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or t.shape[0] != rows or t.stride(1) != 1 or t.shape[1] < n:
        raise ValueError(f"{name} must be [{rows}, >= {n}] with unit column stride, got "
                         f"{tuple(t.shape)} strides {t.stride()}")


_BUILD_DIGEST = None


def build_digest() -> str:
    """Hash of what the library is built from: the HIP sources and headers
    (comments and blank space removed) and the compiler flags.  Tuned launch
    shapes are kept per build: a change of the kernels invalidates them, a
    rebuild of the same sources does not."""
    global _BUILD_DIGEST
    if _BUILD_DIGEST is None:
        from . import build as B
        h = hashlib.sha256()
        paths = sorted(os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC) if f.endswith((".hip", ".h")))
        for path in paths + [os.path.join(B.INCLUDE, "potato.h")]:
            with open(path) as f:
                text = f.read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
            h.update(os.path.basename(path).encode())
            h.update("".join(text.split()).encode())
        h.update(" ".join(B.HIP_FLAGS).encode())
        _BUILD_DIGEST = h.hexdigest()[:16]
    return _BUILD_DIGEST


def autotune_cached(path: str, key: str, run) -> dict:
    """The launch shape stored under ``key`` in the JSON file ``path``, or
    ``run()``'s result, which is then stored there (written to a temporary
    file and renamed, so a reader never sees a partial file).  An unreadable
    file counts as empty."""
    try:
        with open(path) as f:
            table = json.load(f)
        if not isinstance(table, dict):
            table = {}
    except (OSError, ValueError):
        table = {}
    hit = table.get(key)
    if isinstance(hit, dict) and {"block", "steps_per_launch", "grid_blocks"} <= hit.keys():
        return {k: int(hit[k]) for k in ("block", "steps_per_launch", "grid_blocks")}
    result = run()
    table[key] = result
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return result


class Simulator:
    """One context of the simulator: a type table, limits and a launch policy.

    types: list of dicts with the fields of potato_type_params (mass, Ixx,
    Iyy, Izz, arm, alpha, k_f, k_m, tau_m, drag, w_max, w_ref, gains[9],
    budget); glob: dict of controller limits; mode: 0 open loop, 1 closed.
    """

    def __init__(self, types, glob, mode: int, form: str = "fused", block: int = 0,
                 steps_per_launch: int = 0, grid_blocks: int = 0, use_graph: bool = False,
                 debug: bool = False):
        self._lib = L.load()
        self.debug = bool(debug)
        self.n_types = len(types)
        self.mode = int(mode)
        self._types = L.make_type_params(types)
        self._limits = L.make_limits(glob)
        self.opts = self._options(form, block, steps_per_launch, grid_blocks, use_graph)
        h = C.c_void_p()
        L.check(self._lib.potato_create(C.byref(h), C.addressof(self._types), self.n_types,
                                        C.byref(self._limits), C.byref(self.opts)))
        self._h = h

    def _options(self, form, block, steps_per_launch, grid_blocks, use_graph):
        forms = {"auto": L.FORM_AUTO, "plain": L.FORM_PLAIN, "fused": L.FORM_FUSED}
        return L.Options(self.mode, forms[form], int(block), int(steps_per_launch),
                         int(grid_blocks), int(bool(use_graph)))

    def set_options(self, form="fused", block=0, steps_per_launch=0, grid_blocks=0, use_graph=False):
        self.opts = self._options(form, block, steps_per_launch, grid_blocks, use_graph)
        L.check(self._lib.potato_set_options(self._h, C.byref(self.opts)))

    def close(self):
        # pipes use the context: they go first
        for ref in getattr(self, "_pipes", []):
            pipe = ref()
            if pipe is not None:
                pipe.close()
        self._pipes = []
        if getattr(self, "_h", None):
            self._lib.potato_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument structs -------------------------------------------------
    @staticmethod
    def _check_mask(name, t, n):
        if t is not None and (not t.is_cuda or t.dtype != torch.uint8 or t.dim() != 1
                              or t.shape[0] < n or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous device uint8 tensor of length >= n")

    def _structs(self, state, n, type_idx, perm, gains, motor_cmd, wp, resample_every, step0,
                 alive=None, carry=None):
        _check_rows("state", state, N_ROWS, n)
        _check_rows("carry", carry, N_CARRY, n)
        ld = state.stride(0)
        if type_idx is not None:
            if not type_idx.is_cuda or type_idx.dtype != torch.uint8 or type_idx.dim() != 1 \
                    or type_idx.shape[0] < n or not type_idx.is_contiguous():
                raise ValueError("type_idx must be a contiguous device uint8 tensor of length >= n")
            # the device reads an index >= n_types as the last type; debug
            # mode reports it instead (syncs)
            if self.debug and int(type_idx[:n].max().item()) >= self.n_types:
                raise ValueError("type_idx holds an index >= n_types")
        if perm is not None:
            if not perm.is_cuda or perm.dtype != torch.int32 or perm.shape[0] < n or not perm.is_contiguous():
                raise ValueError("perm must be a contiguous device int32 tensor of length >= n")
            # the device clamps entries to [0, n); debug mode checks that the
            # order is a permutation (syncs)
            if self.debug and not torch.equal(torch.sort(perm[:n]).values,
                                              torch.arange(n, dtype=torch.int32, device=perm.device)):
                raise ValueError("perm is not a permutation of 0..n-1")
        _check_rows("gains", gains, 9, n)
        _check_rows("motor_cmd", motor_cmd, 4, n)
        cmd_ld = ld
        n_epochs = 0
        if motor_cmd is not None:
            cmd_ld = motor_cmd.stride(0)
        if wp is not None:
            if not wp.is_cuda or wp.dtype != torch.float32 or wp.dim() != 3 or wp.shape[1] != 3 \
                    or not wp.is_contiguous() or wp.shape[2] < n:
                raise ValueError("wp must be a contiguous device float32 tensor [E, 3, >= n]")
            n_epochs = wp.shape[0]
            if motor_cmd is not None and motor_cmd.stride(0) != wp.shape[2]:
                raise ValueError("motor_cmd and wp must share their row stride")
            cmd_ld = wp.shape[2]
        st = _state(state, carry)
        self._check_mask("alive", alive, n)
        pp = L.Params(_ptr(type_idx), _ptr(perm), _ptr(gains), gains.stride(0) if gains is not None else 0,
                      _ptr(alive))
        cm = L.Cmds(_ptr(motor_cmd), _ptr(wp), n_epochs, int(resample_every), cmd_ld, int(step0))
        return st, pp, cm

    def step(self, state, n_steps, dt, *, n_agents=None, type_idx=None, perm=None, gains=None,
             motor_cmd=None, wp=None, resample_every=0, step0=0, ckpt=None, ckpt_every=0,
             alive=None, carry=None, stream=None):
        """Advance ``state`` ([30, ld] float32, in place) by n_steps steps.
        ``carry`` ([10, ld] float32, in place, optional): the rounding carries
        of position, velocity, cost and position-loop integral (zeros for a
        fresh state); without it the updates are uncompensated.  ``alive``
        (uint8 [n], optional): agents with 0 are not advanced.  ``ckpt``
        ([slots, 40, ld], needs ``carry``) receives the state and carries
        every ``ckpt_every`` steps."""
        n = int(n_agents if n_agents is not None else state.shape[1])
        st, pp, cm = self._structs(state, n, type_idx, perm, gains, motor_cmd, wp,
                                   resample_every, step0, alive, carry)
        if ckpt is not None:
            slots = -(-int(n_steps) // int(ckpt_every)) if ckpt_every > 0 else 0
            if not ckpt.is_cuda or ckpt.dtype != torch.float32 or not ckpt.is_contiguous() \
                    or ckpt.numel() < slots * N_CKPT * st.ld:
                raise ValueError(f"ckpt must be a contiguous device float32 tensor of >= "
                                 f"{slots} x {N_CKPT} x {st.ld} elements")
        L.check(self._lib.potato_step(self._h, C.byref(st), C.byref(pp), C.byref(cm), float(dt),
                                      n, int(n_steps), _ptr(ckpt), int(ckpt_every),
                                      _stream_handle(stream)))
        return state

    def autotune(self, state, dt, probe_steps=200, *, n_agents=None, type_idx=None, perm=None,
                 gains=None, motor_cmd=None, wp=None, resample_every=0, step0=0, carry=None,
                 ckpt_every=0, stream=None, cache=None):
        """Time the fused form's launch shapes on a scratch copy; keep the best.
        ``ckpt_every`` > 0 tunes the variant that writes checkpoints (the
        forward of step_backward's rollouts).

        ``cache`` (default: the POTATO_AUTOTUNE_CACHE environment variable) is
        a JSON file of earlier results, keyed by device, build (build_digest),
        variant, agent count and probe length; a hit skips the timing."""
        n = int(n_agents if n_agents is not None else state.shape[1])
        st, pp, cm = self._structs(state, n, type_idx, perm, gains, motor_cmd, wp,
                                   resample_every, step0, carry=carry)

        self.tuned_from_cache = True

        def run():
            self.tuned_from_cache = False
            best = L.Options()
            L.check(self._lib.potato_autotune(self._h, C.byref(st), C.byref(pp), C.byref(cm),
                                              float(dt), n, int(probe_steps), int(ckpt_every), C.byref(best),
                                              _stream_handle(stream)))
            return dict(block=best.block, steps_per_launch=best.steps_per_launch,
                        grid_blocks=best.grid_blocks)

        path = cache if cache is not None else os.environ.get("POTATO_AUTOTUNE_CACHE")
        if not path:
            return run()
        props = torch.cuda.get_device_properties(state.device)
        key = "|".join(str(x) for x in (
            getattr(props, "gcnArchName", props.name), build_digest(), self.mode, self.n_types,
            type_idx is not None, gains is not None, perm is not None, carry is not None, n,
            int(probe_steps)) + ((f"ckpt{int(ckpt_every)}",) if ckpt_every else ()))
        return autotune_cached(path, key, run)

    def step_backward(self, ckpt, ckpt_every, n_steps, dt, grad_final, *, n_agents=None,
                      type_idx=None, perm=None, gains=None, wp=None, resample_every=0, step0=0,
                      want_gains=True, workspace=None, alive=None, stream=None):
        """Reverse sweep of a checkpointed closed-loop step() call.

        grad_final: [30, ld] cotangent of the final state.  Returns
        (grad_x0 [30, ld], grad_gains [9, ld] or None): rows 0-16 of grad_x0
        are the library's grad_x0 (the initial rigid-body and rotor state),
        rows 17-29 its grad_mem (controller memory and cost)."""
        _check_rows("grad_final", grad_final, 30, n_agents or grad_final.shape[1])
        if not grad_final.is_contiguous():
            raise ValueError("grad_final must be contiguous")
        ld = grad_final.shape[1]
        n = int(n_agents if n_agents is not None else ld)
        if int(ckpt_every) < 1:
            raise ValueError("ckpt_every must be >= 1")
        if not ckpt.is_cuda or ckpt.dtype != torch.float32 or not ckpt.is_contiguous():
            raise ValueError("ckpt must be a contiguous device float32 tensor")
        slots = -(-int(n_steps) // int(ckpt_every))
        if ckpt.numel() < slots * N_CKPT * ld:
            raise ValueError(f"ckpt must hold {slots} x {N_CKPT} x {ld} floats")
        self._check_mask("alive", alive, n)
        pp = L.Params(_ptr(type_idx), _ptr(perm), _ptr(gains),
                      gains.stride(0) if gains is not None else 0, _ptr(alive))
        if wp is None or wp.dim() != 3 or not wp.is_contiguous():
            raise ValueError("wp must be a contiguous device float32 tensor [E, 3, >= n]")
        cm = L.Cmds(None, _ptr(wp), wp.shape[0], int(resample_every), wp.shape[2], int(step0))
        nbytes = int(self._lib.potato_backward_workspace_bytes(self._h, C.byref(pp), n, int(ckpt_every)))
        if nbytes < 0:
            raise ValueError("invalid arguments for potato_backward_workspace_bytes")
        if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=grad_final.device)
        gx0 = torch.empty((30, ld), dtype=torch.float32, device=grad_final.device)
        # the kernel writes every agent's gain cotangent (zero for dead
        # agents); only columns past n_agents need the fill
        alloc = torch.empty if n == ld else torch.zeros
        gg = alloc((9, ld), dtype=torch.float32, device=grad_final.device) if want_gains else None
        L.check(self._lib.potato_step_backward(self._h, C.byref(pp), C.byref(cm), float(dt), n,
                                               int(n_steps), _ptr(ckpt), int(ckpt_every), ld,
                                               _ptr(grad_final), _ptr(gx0), _ptr(gx0[17:]), _ptr(gg),
                                               _ptr(workspace), nbytes, _stream_handle(stream)))
        return gx0, gg

    def detect_collisions(self, state, alive, *, n_agents=None, type_idx=None, died=None,
                          workspace=None, stream=None):
        """Mark colliding agents dead in ``alive`` (uint8 [n], in place).
        ``died`` (int64 device scalar, optional) is incremented by the count."""
        n = int(n_agents if n_agents is not None else state.shape[1])
        _check_rows("state", state, N_ROWS, n)
        self._check_mask("alive", alive, n)
        self._check_mask("type_idx", type_idx, n)
        if died is not None and (not died.is_cuda or died.dtype != torch.int64 or died.numel() < 1):
            raise ValueError("died must be a device int64 tensor")
        nbytes = int(self._lib.potato_collision_workspace_bytes(n))
        if nbytes < 0:
            raise ValueError("invalid agent count")
        if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=state.device)
        st = _state(state, None)
        pp = L.Params(_ptr(type_idx), None, None, 0, None)
        L.check(self._lib.potato_detect_collisions(self._h, C.byref(st), C.byref(pp), n, _ptr(alive),
                                                   _ptr(died), _ptr(workspace), nbytes,
                                                   _stream_handle(stream)))
        return alive

    def count_nonfinite(self, state, *, n_agents=None, count=None, stream=None):
        """Device int64 scalar: agents whose integrated rows hold NaN or Inf
        (added to ``count`` when given)."""
        n = int(n_agents if n_agents is not None else state.shape[1])
        _check_rows("state", state, N_ROWS, n)
        if count is None:
            count = torch.zeros(1, dtype=torch.int64, device=state.device)
        elif not count.is_cuda or count.dtype != torch.int64 or count.numel() < 1:
            raise ValueError("count must be a device int64 tensor")
        st = _state(state, None)
        L.check(self._lib.potato_count_nonfinite(self._h, C.byref(st), n, _ptr(count), _stream_handle(stream)))
        return count

    def order_by_type(self, type_idx, stream=None):
        """Processing order grouping agents by type, longest step budget first."""
        n = type_idx.shape[0]
        nbytes = int(self._lib.potato_order_workspace_bytes(n, self.n_types))
        if nbytes < 0:
            raise ValueError("invalid size for potato_order_workspace_bytes")
        ws = torch.empty(max(nbytes, 4), dtype=torch.uint8, device=type_idx.device)
        perm = torch.empty(n, dtype=torch.int32, device=type_idx.device)
        L.check(self._lib.potato_order_by_type(self._h, _ptr(type_idx), n, _ptr(perm), _ptr(ws),
                                               nbytes, _stream_handle(stream)))
        return perm


class Pipe:
    """Command ingress and position snapshots around running rollouts.

    ``push(cmd)`` uploads the next commands (numpy float32 [3, n] waypoints
    in closed loop, [4, n] rotor commands relative to w_ref in open loop)
    on the pipe's own stream while earlier runs execute; ``run(...)``
    advances the state with the last pushed commands and streams positions
    every ``snap_every`` steps to ``snaps`` (a pinned host float32 tensor
    [n_steps // snap_every, 3, n]) on another stream.  Everything the pipe
    needs is allocated here, once.
    """

    def __init__(self, sim: Simulator, n_agents: int):
        self._lib = sim._lib
        self.sim = sim
        self.n = int(n_agents)
        self.rows = 3 if sim.mode == L.CLOSED_LOOP else 4
        self.n_snaps = 0
        h = C.c_void_p()
        L.check(self._lib.potato_pipe_create(sim._h, self.n, C.byref(h)))
        self._h = h
        sim._pipes = [r for r in getattr(sim, "_pipes", []) if r() is not None] + [weakref.ref(self)]

    def push(self, cmd):
        import numpy as np
        a = np.ascontiguousarray(cmd, dtype=np.float32)
        if a.shape != (self.rows, self.n):
            raise ValueError(f"commands must be [{self.rows}, {self.n}], got {a.shape}")
        L.check(self._lib.potato_pipe_push(self._h, a.ctypes.data_as(C.c_void_p)))

    def run(self, state, n_steps, dt, *, snap_every=0, snaps=None, type_idx=None, perm=None,
            gains=None, alive=None, carry=None, stream=None):
        _check_rows("state", state, N_ROWS, self.n)
        due = int(n_steps) // int(snap_every) if snap_every > 0 else 0
        if due:
            if snaps is None or snaps.is_cuda or snaps.dtype != torch.float32 \
                    or not snaps.is_contiguous() or snaps.numel() < due * 3 * self.n:
                raise ValueError(f"snaps must be a contiguous host float32 tensor of >= {due} x 3 x {self.n}")
        st, pp, _ = self.sim._structs(state, self.n, type_idx, perm, gains, None, None, 0, 0, alive,
                                      carry)
        L.check(self._lib.potato_pipe_run(self._h, C.byref(st), C.byref(pp), float(dt), int(n_steps),
                                          int(snap_every), _ptr(snaps) if due else None,
                                          _stream_handle(stream)))
        self.n_snaps += due
        return state

    def wait_snapshots(self, count):
        L.check(self._lib.potato_pipe_wait_snapshots(self._h, int(count)))

    def sync(self):
        L.check(self._lib.potato_pipe_sync(self._h))

    def stats(self):
        """(snapshots enqueued, of which written directly to pinned host memory)."""
        total, direct = C.c_int64(0), C.c_int64(0)
        L.check(self._lib.potato_pipe_stats(self._h, C.byref(total), C.byref(direct)))
        return total.value, direct.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.potato_pipe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
