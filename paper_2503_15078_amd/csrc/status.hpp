// Error codes and the thread-local last-error message shared by the library's
// translation units.
#pragma once
#include <string>

#include "lgsim.h"

namespace lg {
void set_error(const std::string& msg);
const char* last_error();
}  // namespace lg
