// Helpers of the extern "C" boundary: no C++ exception crosses it; internal
// errors become ts_status codes plus the thread-local message.
#pragma once
#include <exception>

#include "problem.h"

#define TS_API_BEGIN try {
#define TS_API_END                                   \
  }                                                  \
  catch (const tsmg::Error& e) {                     \
    tsmg::set_error(e.msg);                          \
    return e.code;                                   \
  }                                                  \
  catch (const std::exception& e) {                  \
    tsmg::set_error(e.what());                       \
    return TS_EDEVICE;                               \
  }                                                  \
  catch (...) {                                      \
    tsmg::set_error("unknown internal error");       \
    return TS_EDEVICE;                               \
  }
