// abi_guard.hpp -- keeps C++ exceptions from crossing the C ABI.
//
// Every extern "C" entry point that returns mxl_status is written as a
// function-try-block whose handler is
//     catch (...) { return mxl::abi_exception(__func__); }
// so a std::bad_alloc from host-side work (level sets, per-block tables,
// std::vector growth, handle allocation) becomes MXL_ERR_OUT_OF_MEMORY and
// any other exception MXL_ERR_INTERNAL, with mxl_last_error() naming the
// entry point.  The last-error text lives in a fixed thread-local buffer, so
// recording an error never allocates and cannot throw.
//
// Host-only standard C++: this header is also compiled by g++ in the CPU
// tests of the guard.
#pragma once

#include <cstdio>
#include <cstring>
#include <exception>
#include <new>

#include "../../include/mxl.h"

namespace mxl {

constexpr size_t kErrCap = 512;

inline char *error_buffer() noexcept {
    thread_local char buf[kErrCap] = {0};
    return buf;
}

// Stores msg (truncated to the buffer) as this thread's last error.
inline mxl_status record_error(mxl_status st, const char *msg) noexcept {
    char *buf = error_buffer();
    if (!msg) msg = "";
    size_t n = std::strlen(msg);
    if (n >= kErrCap) n = kErrCap - 1;
    std::memcpy(buf, msg, n);
    buf[n] = '\0';
    return st;
}

inline const char *last_error() noexcept { return error_buffer(); }

// Maps the exception being handled to a status; call only from a handler.
inline mxl_status abi_exception(const char *entry) noexcept {
    char msg[kErrCap];
    mxl_status st = MXL_ERR_INTERNAL;
    try {
        throw;
    } catch (const std::bad_alloc &) {
        st = MXL_ERR_OUT_OF_MEMORY;
        std::snprintf(msg, sizeof msg, "%s: host memory allocation failed", entry);
    } catch (const std::exception &e) {
        std::snprintf(msg, sizeof msg, "%s: internal error: %s", entry, e.what());
    } catch (...) {
        std::snprintf(msg, sizeof msg, "%s: internal error (unknown exception)", entry);
    }
    return record_error(st, msg);
}

}  // namespace mxl
