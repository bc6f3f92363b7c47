// Library-wide error reporting: one thread-local message for the last failure.
#pragma once
#include <string>

namespace thcsox {
int set_error(int code, const std::string& msg);   // stores msg, returns code
void clear_error();
}  // namespace thcsox
