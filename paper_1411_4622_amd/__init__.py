"""MI355X (gfx950) simulated annealing tomography with a pre-calculated
intersection lengths array (PILA): Python binding of libpila.so.

Entry points mirror the C ABI in include/pila.h: pila_build, pila_forward,
pila_backproject, sat_run, sat_run_static, sat_run_batch, the chain graphs
(sat_graph, sat_batch_graph), sirt_run, sirt_seq_run, sat_drt_run, the srv_*
server (Server), device_info.
"""
from ._binding import (EXPORTED, LIB_PATH, PILA_F32, PILA_F64, Geometry, Graph, Job, Pila, PilaError,
                       SatParams, Server, device_info, last_error, load, pila_backproject, pila_build,
                       pila_forward, sat_batch_graph, sat_graph, sat_run, sat_run_batch, sat_run_static,
                       sat_workspace, sat_drt_run, sirt_run, sirt_seq_run)

__all__ = ["EXPORTED", "LIB_PATH", "PILA_F32", "PILA_F64", "Geometry", "Graph", "Job", "Pila", "PilaError",
           "SatParams", "Server", "device_info", "last_error", "load", "pila_backproject", "pila_build",
           "pila_forward", "sat_batch_graph", "sat_graph", "sat_run", "sat_run_batch", "sat_run_static",
           "sat_workspace", "sat_drt_run", "sirt_run", "sirt_seq_run"]
