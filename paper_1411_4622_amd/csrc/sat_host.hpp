// Host helpers shared by the chain entry points (sat_run, sat_run_batch) and
// the server: workspace layout, argument checks, chain descriptors, launch
// limits.
#pragma once

#include <cstddef>

#include "sat_chain.hpp"

namespace pila {

size_t align256(size_t x);
// device bytes of one chain's state: residual, tile sums and drifts, carry, stats
size_t chain_bytes(const pila_geom* g, const sat_params* p);
int32_t check_params(const pila_geom* g, const pila_csr* c, const sat_params* p);
// descriptor of one chain whose state lives at ws (chain_bytes bytes)
ChainJob make_job(const pila_geom* g, const pila_csr* c, const double* sino, const sat_params* p,
                  double* image, char* ws);
int device_props(hipDeviceProp_t* prop);
// whether the pipelined body's index arithmetic holds for this PILA
bool piped_allowed(const pila_geom* g, const pila_csr* c);
// LDS bytes of a pipelined chain with the residual partly in LDS; sets J->UL
int64_t hybrid_lds(ChainJob* J, int64_t budget);
// row entries per lane in registers of the long-row body (64 kLongE per
// row); up to kLongOver more per lane are read in place
constexpr int kLongE = 16;
constexpr int kLongOver = 8;
// whether the long-row body takes this chain (one estimate per wavefront)
bool long_allowed(const pila_geom* g, const pila_csr* c, const sat_params* p);
// LDS bytes of a long-row chain with the residual partly in LDS; sets J->UL
int64_t long_lds(ChainJob* J, int64_t budget);
int32_t set_lds(const void* k, int bytes);
// the slot words of a PILA's nnz entries for the pipelined body in global
// mode, for J's LDS layout (J.UL set), written to dst on stream st
int32_t launch_tcol(const ChainJob& J, int64_t nnz, int32_t* dst, hipStream_t st);

// pila_build with a caller-supplied device scratch of pila_build_scratch(geom) bytes
size_t pila_build_scratch(const pila_geom* geom);
int32_t pila_build_with(const pila_geom* geom, pila_csr* csr, void* d_scratch, hipStream_t st);

}  // namespace pila
