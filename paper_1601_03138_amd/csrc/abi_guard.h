// No C++ exception crosses the C ABI (include/fdx.h).  Every entry point whose body can
// allocate host memory (std::vector, std::string) runs that body between FDX_ABI_TRY and
// FDX_ABI_CATCH(ctx): std::bad_alloc becomes FDX_ENOMEM, any other exception FDX_EINVAL, and
// the message goes to the context's fixed-size last-error buffer (writing it allocates
// nothing, so the handler itself cannot throw).
#pragma once

#include <cstddef>
#include <cstdio>
#include <exception>
#include <new>

#include "../../include/fdx.h"

namespace fdx {

// Status code and message of the exception in flight.  Call only from inside a catch block:
// it rethrows the current exception to inspect it.  err may be null.
inline int classify_exception(char *err, size_t len) noexcept {
    try {
        throw;
    } catch (const std::bad_alloc &) {
        if (err && len) std::snprintf(err, len, "host memory allocation failed");
        return FDX_ENOMEM;
    } catch (const std::exception &e) {
        if (err && len) std::snprintf(err, len, "internal error: %s", e.what());
        return FDX_EINVAL;
    } catch (...) {
        if (err && len) std::snprintf(err, len, "internal error: unknown exception");
        return FDX_EINVAL;
    }
}

}  // namespace fdx

#define FDX_ABI_TRY try {
#define FDX_ABI_CATCH(ctx)                                                                    \
    }                                                                                         \
    catch (...) {                                                                             \
        return ::fdx::abi_exception(ctx);                                                     \
    }
