"""MI355X (gfx950) implementation of the per-day hot path of the event-based
epidemic framework of Bauer, Engblom & Widgren (arXiv:1502.02908): SSA per
node, scheduled events in dependency levels, and the phi update, behind the C
ABI declared in include/episim.h."""
from .sim import (EVENTS_LEVELS, EVENTS_SERIAL, LAUNCH_KERNELS, LAUNCH_PERSISTENT,  # noqa: F401
                  SIM_EDEVICE, SIM_EINFEASIBLE, SIM_EINVAL, SIM_ELIMIT, SIM_ENOMEM, SIM_ESTATE, SIM_OK, SimError, Simulator, SlotHandle, lib, plan_levels, workspace_bytes)
