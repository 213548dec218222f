// Thread-local error text behind tsk_last_error().
#pragma once

#include <stdarg.h>
#include <stdio.h>

#include "../../include/tsk.h"

namespace tsk {

char* last_error_buffer();

inline tsk_status fail(tsk_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(last_error_buffer(), 512, fmt, ap);
  va_end(ap);
  return st;
}

}  // namespace tsk
