// dispatch.h -- run a generic lambda with the (lattice, storage, arithmetic)
// types a context is configured for.
#pragma once
#include <type_traits>

#include "ctx.h"
#include "lattice.h"

namespace lbm {

template <class F>
inline hipError_t dispatch(lbm_ctx *c, F &&fn)
{
    if (c->cfg.lattice == LBM_D2Q9) {
        switch (c->cfg.storage) {
        case LBM_F64: return fn(D2Q9{}, StF64{}, double{});
        case LBM_F32: return fn(D2Q9{}, StF32{}, float{});
        case LBM_F16: return fn(D2Q9{}, StF16{}, float{});
        default: return fn(D2Q9{}, StBF16{}, float{});
        }
    }
    switch (c->cfg.storage) {
    case LBM_F64: return fn(D3Q19{}, StF64{}, double{});
    case LBM_F32: return fn(D3Q19{}, StF32{}, float{});
    case LBM_F16: return fn(D3Q19{}, StF16{}, float{});
    default: return fn(D3Q19{}, StBF16{}, float{});
    }
}

} // namespace lbm
