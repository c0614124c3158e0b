// Host stand-in for <hip/hip_runtime.h>, used only by the FLOP-counting build of the
// integrand headers (tests/flopcount/count.cpp): the device qualifiers become plain
// inline functions and the few device builtins the headers call are routed to the
// counting scalar's functions declared by count.cpp before it includes the headers.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __builtin_amdgcn_rcp(x) fc_rcp(x)
#define __builtin_amdgcn_rsq(x) fc_rsq(x)
#define __builtin_amdgcn_bitop3_b32(a, b, c, imm) fc_xor3(a, b, c)
#define VG_OPAQUE_SGPR(x) (void)(x)
// a mathematical function priced at its library cost, its own operations not counted
#define VG_PRICED(kind, x) ::fc::Priced vg_priced_(::fc::price_##kind, (x).u)
// cross-lane builtins of the wave reductions (not on the counted path): one lane
#define __builtin_amdgcn_update_dpp(old, v, ctrl, rmask, bmask, bound) (v)
#define __builtin_amdgcn_readlane(v, lane) (v)
