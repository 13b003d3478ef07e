// Internal helpers of the host side of libinrf: error reporting and small
// utilities shared by the C-ABI entry points.
#pragma once

#include <cstdint>
#include <cstdio>
#include <exception>
#include <string>

#include "inrf.h"

namespace inrf {

// Thread-local message of the last failure (returned by inrf_last_error).
void set_error(const std::string& msg);
void clear_error();

struct Error {
    inrf_status code;
    std::string msg;
};

[[noreturn]] inline void fail(inrf_status code, const std::string& msg) { throw Error{code, msg}; }

// Runs `f`, converting any exception into a status code and message, so that
// nothing crosses the C boundary.
template <class F>
inrf_status guarded(const char* where, F&& f) {
    try {
        clear_error();
        f();
        return INRF_OK;
    } catch (const Error& e) {
        set_error(std::string(where) + ": " + e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error(std::string(where) + ": host out of memory");
        return INRF_E_BUILD;
    } catch (const std::exception& e) {
        set_error(std::string(where) + ": " + e.what());
        return INRF_E_BUILD;
    } catch (...) {
        set_error(std::string(where) + ": unknown failure");
        return INRF_E_BUILD;
    }
}

inline void require(bool ok, const std::string& msg) {
    if (!ok) fail(INRF_E_INVALID, msg);
}

int resolve_threads(int requested);

}  // namespace inrf
